#!/usr/bin/env python3
"""Throughput of the fused split-form SBP + RK4 step on one MI355X.

Default workload: the large single run -- periodic [-50,50]^2 on a 4096 x 4096
grid, random-phase bathymetry (amplitude 0.2) under a still-water level of 1,
a seeded Gaussian surface bump, lambda = 500, g = 9.81, classical RK4 with a
fixed step at CFL 0.5, FP64 state and arithmetic.  A "step" is one RK4 step
over the whole grid (one step kernel on the default fused path; --path selects
the two-kernel pair path or the four-kernel stage path); the value is RK-stage
cell-updates per second, nx * ny * 4 * steps / seconds, with all inputs
resident in HBM before the timed region starts.

The timed region is `--repeats` runs of `--steps` steps each (median
reported), after `--warmup` untimed steps; the HIP graphs the timed calls
replay are instantiated before the first timing event.  The roofline entry
is the step kernel's: the method's 11 values per node and step (88 B in FP64)
over the mean launch duration in the timed region, against the 8 TB/s HBM
peak, with the FP64 arithmetic rate beside it.

The same run is repeated with reflecting walls and with FP32 storage and
arithmetic (energy and mass still reduced in FP64), reported under
"variants".  Each 4096^2 run's mass and energy after --drift-steps steps are
compared with the FP64 oracle's over the same steps (each side initializes
the workload itself).  The CPU oracle is timed on the host as a baseline: its
threaded build on every usable core and its serial build on one.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RK-stage cell-updates/s and % HBM peak (FP64 vs FP32); adjoint:forward cost"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM traffic of one RK4 step, in values per node, and kernel
# launches per step, for each step path:
#  pairs:  pair 1 reads q, b and writes acc, Yb (16); pair 2 reads Yb, b, q, acc
#          and writes q_new (21)  -> 37 values, 2 launches
#  stages: stage 1 reads q, b and writes acc, Y (16); stages 2 and 3 read Y, b,
#          q, acc and write acc, Y (26 each); stage 4 reads Y, b, acc and writes
#          q (16)                 -> 84 values, 4 launches
#  fused:  the step kernel reads q, b and writes q_new -> 11 values, 1 launch
PATHS = {"pairs": (37, 2), "stages": (84, 4), "fused": (11, 1)}
# Arithmetic of one node and step as the kernels implement it, excluding the
# step kernel's redundant ring evaluations: 4 right-hand sides of 178 flops
# (56 for the 24 differences and the products they need, 12 for the node's own
# products and constants, 9 for h_t, 33 each for the u and v rows, 17 for the
# w-row fluxes, 5 for dividing the u, v, w rows by h, 12 for eta_t, 1 for the
# reciprocal of h) and the stage updates (3 x 20 + 10).  Each add, multiply or
# reciprocal counts 1, a fused multiply-add 2.
FLOPS_PER_NODE_STEP = 4 * 178 + 70
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Untimed steps before the variants' timed runs (on a copy of the state): after an
# idle spell of a few tens of ms the GPU runs the next ~30 launches up to 30%
# slower while its clocks settle.
SETTLE_STEPS = 64
# Device memory the adjoint variant may fill with the stage states of the rollout's last
# steps (beside its run that recomputes every step).
ADJOINT_STORE_CAP_BYTES = 240 * 2**30
# HBM traffic of the step kernel on the default workload (4096^2 periodic FP64,
# its default 32 x 24 tiles), from the FETCH_SIZE and WRITE_SIZE passes
# summarized in profiles/step_kernel_random_phase_4096_periodic_f64.md
# (FETCH_SIZE scaled by 1.99992 and WRITE_SIZE by 1.0, the factors a plain
# 1 GiB copy reads): bytes per node and launch.  Reported only while the kernel
# sources hash to the value they had when the counters were taken (or to a later
# version whose step kernel assembles to the same instructions: the relaxed-input
# mode of the step tile added other instantiations only).
STEP_TRAFFIC_BYTES_PER_NODE = (1082889614.0 + 671088640.0) / 16777216
STEP_KERNEL_SOURCES = ("sgn_common.hpp", "sgn_stage.hpp", "sgn_mms.hpp", "sgn_pair.hpp", "sgn_reduce.hpp",
                       "sgn_fused.hpp")
STEP_SOURCES_SHA256 = "4e8c6d844ce4d6910838e883f1ad1701f29b44e44029454f19aa51055cbf82fb"
KERNELS = {"pairs": "pair_kernel (two fused RK4 stages; mean over the 2 launches of a step)",
           "stages": "stage_kernel (fused RHS + RK4 stage; mean over the 4 launches of a step)",
           "fused": "step_kernel (one whole RK4 step per launch)"}
ALL_VARIANTS = {"f32", "reflecting", "ensemble", "small", "adjoint", "paths", "paper", "relaxation", "totals",
                "adaptive", "longdrift"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def lake_at_rest_energy(grid, b, mass):
    """Energy of the lake at rest holding the same mass: g/2 sum M (H^2 - b^2),
    H = (mass + sum M b) / sum M (the datum of the potential energy is b)."""
    import numpy as np
    wx = np.full(grid.nx, grid.spacing()[0])
    wy = np.full(grid.ny, grid.spacing()[1])
    if grid.bc_x == 1:
        wx[0] *= 0.5
        wx[-1] *= 0.5
    if grid.bc_y == 1:
        wy[0] *= 0.5
        wy[-1] *= 0.5
    M = np.outer(wy, wx)
    H = (mass + (M * b).sum()) / M.sum()
    return 0.5 * grid.g * (M * (H * H - b * b)).sum()


def run_gpu(problem, dtype, steps, warmup, label, path="pairs", tile_y=None, repeats=1, drift_steps=0, settle=0):
    """Times `repeats` runs of `steps` RK4 steps (after `warmup` untimed ones) with
    HIP events on the solver's stream; every graph a timed call replays is
    instantiated before the first event.  With drift_steps > 0, also records
    mass and energy over the first drift_steps steps from the initial state
    (step kernel epilogue) for the comparison with the oracle.  With settle > 0
    (the variants, not the headline run), `settle` more untimed steps run on a
    copy of the state just before the first timed run, so that the clocks have
    left the idle spell behind; the state's own trajectory is unchanged."""
    import numpy as np
    import torch
    from paper_2601_02540_amd.binding import Solver

    grid = problem.grid
    s = Solver(grid, dtype)
    s.set_step_path(path)
    if tile_y is not None:
        s.set_tile_y(tile_y)
    values, launches = PATHS[path]
    b = torch.from_numpy(problem.b).to(dtype).cuda().contiguous()
    q = torch.from_numpy(problem.q0).to(dtype).cuda().contiguous()
    s.set_bathymetry(b)
    s.init_aux(q)
    dt = s.cfl_dt(q, 0.5)
    m0, e0 = s.mass_energy(q)
    series = None
    if drift_steps > 0:
        qd = q.clone()
        series = s.step_totals(qd, dt, drift_steps).cpu().numpy()
        del qd
    log(f"[{label}] dt={dt:.6e} warmup={warmup} repeats={repeats}")
    s.prepare_step(q, dt, warmup)
    s.prepare_step(q, dt, steps)
    if warmup > 0:
        s.step(q, dt, warmup)
    if settle > 0:
        qs = q.clone()
        s.profile_stages(qs, dt, settle)
        del qs
    torch.cuda.synchronize()
    stream = s.stream
    secs = []
    t = warmup * dt
    for _ in range(repeats):
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start.record(stream)
        s.step(q, dt, steps, t0=t)
        t_end.record(stream)
        t_end.synchronize()
        torch.cuda.synchronize()
        secs.append(t_start.elapsed_time(t_end) / 1e3)
        t += steps * dt
    sec = float(np.median(secs))
    # per-launch durations of the path's kernels (direct launches, events bound to the step kernel or
    # between the kernels of the other paths), after an unrecorded pass of 64 steps: after an idle spell
    # of a few tens of ms the GPU runs the next ~30 launches up to 30% slower while its clocks settle
    s.profile_stages(q, dt, 64)
    ms = s.profile_stages(q, dt, 16)
    s.check()
    m1, e1 = s.mass_energy(q)
    cells = grid.nx * grid.ny
    esize = 8 if dtype == torch.float64 else 4
    launch_s = sec / (launches * steps)
    achieved = values / launches * esize * cells / launch_s / 1e9
    e_rest = lake_at_rest_energy(grid, problem.b.astype(np.float64), m0)
    res = {
        "value": cells * 4 * steps / sec,
        "sec": sec,
        "ms_per_step": sec / steps * 1e3,
        "ms_per_step_repeats": [x / steps * 1e3 for x in secs],
        "repeats": repeats,
        "dt": dt,
        "stage_launch_us": launch_s * 1e6,
        "achieved_GBs": achieved,
        "frac": achieved / HBM_PEAK_GBS,
        "path": path,
        "tile_y": tile_y,
        "kernel_ms": ({"pair1": ms[0], "pair2": ms[1]} if path == "pairs" else
                      {"step": ms[0]} if path == "fused" else
                      {"stage1": ms[0], "stage2": ms[1], "stage3": ms[2], "stage4": ms[3]}),
        "mass_drift_rel": (m1 - m0) / abs(m0),
        "energy_drift_rel": (e1 - e0) / abs(e0),
        "energy_drift_rel_to_excess": (e1 - e0) / abs(e0 - e_rest),
        "energy_final": e1,
        "steps_total": warmup + repeats * steps,
    }
    if series is not None:
        res["drift_series"] = {"steps": drift_steps, "mass0": m0, "energy0": e0,
                               "mass": float(series[-1, 0]), "energy": float(series[-1, 1])}
    log(f"[{label}] {res['value']:.4e} cell-stage/s  {res['ms_per_step']:.3f} ms/step (median of {repeats})  "
        f"{achieved:.0f} GB/s ({100 * res['frac']:.1f}% of HBM peak)  dE/E={res['energy_drift_rel']:.3e}")
    s.close()
    del q, b
    torch.cuda.empty_cache()
    return res


def run_ensemble(count, steps, warmup, dtype, label, path="fused"):
    """The ensemble workload: `count` instances of seeded sizes and boundaries in one batch."""
    import numpy as np
    import torch
    from paper_2601_02540_amd import workloads as W
    from paper_2601_02540_amd.binding import Batch

    t0 = time.perf_counter()
    probs = W.ensemble(count, seed=4)
    log(f"[{label}] generated {count} instances in {time.perf_counter() - t0:.1f} s")
    batch = Batch([p.grid for p in probs], dtype)
    batch.set_step_path(path)
    qs = [torch.from_numpy(p.q0).to(dtype).cuda().contiguous() for p in probs]
    for i, p in enumerate(probs):
        batch.set_bathymetry(i, torch.from_numpy(p.b).to(dtype).cuda().contiguous())
    batch.set_states(qs)
    batch.init_aux()
    dts = batch.cfl_dt(0.5)
    ty, bpc, tune_ms = batch.autotune(dts)
    m0, e0 = batch.mass_energy()
    if warmup > 0:
        batch.step(dts, warmup)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(batch.stream)
    batch.step(dts, steps)
    t_end.record(batch.stream)
    t_end.synchronize()
    sec = t_start.elapsed_time(t_end) / 1e3
    assert batch.check() == -1
    m1, e1 = batch.mass_energy()
    nodes = batch.total_nodes()
    esize = 8 if dtype == torch.float64 else 4
    values, launches = PATHS[path]
    achieved = values * esize * nodes * steps / sec / 1e9
    sizes = sorted({p.grid.nx for p in probs})
    res = {
        "value": nodes * 4 * steps / sec,
        "instances": count,
        "nodes": nodes,
        "sizes": sizes,
        "periodic_instances": sum(1 for p in probs if p.grid.bc_x == 0),
        "steps": steps,
        "ms_per_step": sec / steps * 1e3,
        "achieved_GBs": achieved,
        "frac": achieved / HBM_PEAK_GBS,
        "path": path,
        "autotuned": {"tile_y": ty, "blocks_per_cu": bpc, "step_ms": tune_ms},
        "max_abs_energy_drift_rel": max(abs(b - a) / abs(a) for a, b in zip(e0, e1)),
        "max_abs_mass_drift_rel": max(abs(b - a) / abs(a) for a, b in zip(m0, m1)),
    }
    # two 128^2 instances (one per boundary type) for the comparison with the FP64 oracle
    picks = {}
    for bc in (0, 1):
        i = next((k for k, p in enumerate(probs) if p.grid.bc_x == bc and p.grid.nx == 128), None)
        if i is not None:
            picks[f"ensemble_{i}"] = {"instance": i, "steps": warmup + steps, "mass0": m0[i], "energy0": e0[i],
                                      "mass": m1[i], "energy": e1[i]}
    res["drift_instances"] = picks
    log(f"[{label}] {res['value']:.4e} node-stage/s over {nodes} nodes  {res['ms_per_step']:.3f} ms/step  "
        f"{achieved:.0f} GB/s  tiles ty={ty} bpc={bpc}")
    batch.close()
    del qs
    torch.cuda.empty_cache()
    return res


def run_adjoint(n, steps, label):
    """adjoint:forward cost on the gauge workload: reflecting [0,30]x[0,10], n^2, FP64, 16 gauges,
    loss against the series of a target run; gradient wrt the initial surface and the bathymetry."""
    import numpy as np
    import torch
    from paper_2601_02540_amd import workloads as W
    from paper_2601_02540_amd.binding import SgnError, Solver

    gp = W.gauge_problem(n, seed=5)
    g = gp.grid
    s = Solver(g, torch.float64)
    nodes = torch.from_numpy(gp.gauges[:, 0] * g.nx + gp.gauges[:, 1]).cuda()
    z0 = torch.from_numpy(gp.zeta0).cuda()
    b = torch.from_numpy(gp.b).cuda()
    q = torch.zeros((5, g.ny, g.nx), dtype=torch.float64, device="cuda")
    q[0] = z0 - b
    q[4] = q[0]
    s.set_bathymetry(b)
    dt = s.cfl_dt(q, 0.5)
    s.set_bathymetry(torch.from_numpy(gp.target_b).cuda())
    target = s.gauge_series(torch.from_numpy(gp.target_zeta0).cuda(), steps, dt, nodes)
    s.set_bathymetry(b)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    qf = q.clone()
    s.init_aux(qf)
    s.step(qf, dt, 8)  # warm-up (graph capture)
    t_fwd, _ = timed(lambda: s.step(qf, dt, steps))
    t_series, _ = timed(lambda: s.gauge_series(z0, steps, dt, nodes))
    w = min(20, steps)
    s.gauge_loss_grad(z0, w, dt, nodes, target[:w].contiguous())  # warm-up of the adjoint buffers
    t_grad, (L, gz, gb) = timed(lambda: s.gauge_loss_grad(z0, steps, dt, nodes, target))
    # the same gradient keeping the stage states of the rollout's last steps in free device memory
    # (at most ADJOINT_STORE_CAP_BYTES), so that the reverse sweep recomputes only the others
    state_bytes = 5 * g.nx * g.ny * 8
    free_bytes, _ = torch.cuda.mem_get_info()
    store = int(min(ADJOINT_STORE_CAP_BYTES, 0.8 * free_bytes))
    kept = min(steps, max(0, (store // state_bytes - 1) // 4)) if store >= 5 * state_bytes else 0
    kept_res = {"store_bytes": store, "kept_steps": kept}
    if kept > 0:
        s.set_adjoint_store(store)
        try:
            s.gauge_loss_grad(z0, steps, dt, nodes, target)  # allocates the storage
        except SgnError as e:  # storage not available after all: reported, the rest of the run goes on
            kept_res["error"] = str(e)
            kept = 0
        s.set_adjoint_store(0 if kept == 0 else store)
    if kept > 0:
        t_kept, (L2, gz2, gb2) = timed(lambda: s.gauge_loss_grad(z0, steps, dt, nodes, target))
        kept_res.update({"gradient_s": t_kept, "adjoint_to_forward": t_kept / t_fwd,
                         "same_bits": bool(L2 == L and torch.equal(gz2, gz) and torch.equal(gb2, gb))})
        s.set_adjoint_store(0)
        log(f"[{label}] keeping the stage states of the last {kept} of {steps} steps ({store / 2**30:.0f} GiB): "
            f"gradient {t_kept:.3f} s, adjoint:forward = {t_kept / t_fwd:.2f}, same bits {kept_res['same_bits']}")
    # context: the same forward on the four-stage path (84 values per node and step)
    s.set_step_path("stages")
    qs = q.clone()
    s.init_aux(qs)
    s.step(qs, dt, 8)
    t_fwd4, _ = timed(lambda: s.step(qs, dt, steps))
    s.set_step_path("fused")
    res = {"grid": [g.nx, g.ny], "steps": steps, "gauges": int(len(gp.gauges)), "dt": dt,
           "checkpoint_every": int(np.ceil(np.sqrt(steps))), "loss": L,
           "forward_s": t_fwd, "forward_with_gauges_s": t_series, "gradient_s": t_grad,
           "adjoint_to_forward": t_grad / t_fwd,
           "forward_four_stage_s": t_fwd4, "adjoint_to_four_stage_forward": t_grad / t_fwd4,
           "kept_rollout_tail": kept_res,
           "grad_norms": {"zeta0": float(torch.linalg.norm(gz)), "b": float(torch.linalg.norm(gb))}}
    log(f"[{label}] forward {t_fwd:.3f} s, gradient {t_grad:.3f} s, adjoint:forward = {t_grad / t_fwd:.2f} "
        f"(four-stage forward {t_fwd4:.3f} s: {t_grad / t_fwd4:.2f})")
    s.close()
    torch.cuda.empty_cache()
    return res


def run_paper_setups(path, tile_y):
    """The paper's scaling study (solitary wave over a Gaussian obstacle, nx = 2^n,
    ny = nx/2, run to t = 12 in the paper) and its long-term cylindrical dam break
    (10^8 nodes, run to t = 300).  Fixed-step RK4 at CFL 0.5 here, so the
    projected runtimes (timed steps x steps to the final time) are context for
    the paper's adaptive runs, not a like-for-like comparison."""
    import math
    from paper_2601_02540_amd import workloads as W
    out = {}
    for nx in (1024, 2048, 4096, 8192):
        p = W.gaussian_obstacle(nx)
        r = run_gpu(p, torch_f64(), 100, 8, f"gaussian obstacle {nx}x{nx // 2}", path, tile_y)
        steps_to_end = math.ceil(12.0 / r["dt"])
        out[f"gaussian_obstacle_{nx}x{nx // 2}"] = {
            "value": r["value"], "ms_per_step": r["ms_per_step"], "ms_per_rhs": r["ms_per_step"] / 4,
            "dt": r["dt"], "steps_to_t12": steps_to_end,
            "projected_runtime_to_t12_s": steps_to_end * r["ms_per_step"] / 1e3,
            "energy_drift_rel": r["energy_drift_rel"], "mass_drift_rel": r["mass_drift_rel"]}
    p = W.cylindrical_dam_break(10000, 1100.0)
    r = run_gpu(p, torch_f64(), 100, 8, "cylindrical dam break 10000x10000", path, tile_y)
    steps_to_end = math.ceil(300.0 / r["dt"])
    out["cylindrical_dam_break_10000x10000"] = {
        "value": r["value"], "ms_per_step": r["ms_per_step"], "dt": r["dt"], "steps_to_t300": steps_to_end,
        "projected_runtime_to_t300_s": steps_to_end * r["ms_per_step"] / 1e3,
        "energy_drift_rel": r["energy_drift_rel"], "mass_drift_rel": r["mass_drift_rel"]}
    log(f"[paper setups] dam break projected to t=300: {out['cylindrical_dam_break_10000x10000']['projected_runtime_to_t300_s']:.0f} s")
    return out


def run_long_dam_break(path, tile_y, t_end=300.0):
    """The paper's long-term cylindrical dam break run to the end: 10^8 nodes,
    FP64, [-1100,1100]^2, reflecting, fixed-step RK4 at CFL 0.5 to t = 300.
    Logs progress every 5000 steps."""
    import math
    import numpy as np
    import torch
    from paper_2601_02540_amd import workloads as W
    from paper_2601_02540_amd.binding import Solver
    p = W.cylindrical_dam_break(10000, 1100.0)
    g = p.grid
    s = Solver(g, torch.float64)
    s.set_step_path(path)
    if tile_y is not None:
        s.set_tile_y(tile_y)
    b = torch.from_numpy(p.b).cuda()
    q = torch.from_numpy(p.q0).cuda()
    s.set_bathymetry(b)
    s.init_aux(q)
    dt0 = s.cfl_dt(q, 0.5)
    nsteps = math.ceil(t_end / dt0)
    dt = t_end / nsteps
    m0, e0 = s.mass_energy(q)
    log(f"[long dam break] {nsteps} steps of {dt:.6e} to t = {t_end}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        k = min(5000, nsteps - done)
        s.step(q, dt, k, t0=done * dt)
        s.check()
        done += k
        log(f"[long dam break] {done}/{nsteps} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m1, e1 = s.mass_energy(q)
    e_rest = lake_at_rest_energy(g, p.b, m0)
    eta = q[0, g.ny // 2, g.nx // 2:].cpu().numpy() - 1.0  # surface elevation along the positive x half-axis
    x = g.x_nodes()[g.nx // 2:]
    res = {"nodes": g.nx * g.ny, "steps": nsteps, "dt": dt, "wall_s": wall,
           "node_stage_per_s": g.nx * g.ny * 4 * nsteps / wall,
           "mass_drift_rel": (m1 - m0) / abs(m0), "energy_drift_rel": (e1 - e0) / abs(e0),
           "energy_drift_rel_to_excess": (e1 - e0) / abs(e0 - e_rest),
           "max_surface_elevation_on_axis": float(eta.max()),
           "x_of_max_elevation": float(x[int(np.argmax(eta))])}
    log(f"[long dam break] {wall:.1f} s, dE/(E - E_rest) = {res['energy_drift_rel_to_excess']:.3e}")
    s.close()
    return res


def run_relaxation(problem, steps, warmup, path, tile_y):
    """Relaxation RK4 on the main workload: throughput and energy drift, against
    classical RK4 over the same steps from the same state."""
    import torch
    from paper_2601_02540_amd.binding import Solver
    grid = problem.grid
    s = Solver(grid, torch.float64)
    s.set_step_path(path)
    if tile_y is not None:
        s.set_tile_y(tile_y)
    b = torch.from_numpy(problem.b).cuda()
    q = torch.from_numpy(problem.q0).cuda()
    s.set_bathymetry(b)
    s.init_aux(q)
    dt = s.cfl_dt(q, 0.5)
    q_plain = q.clone()
    _, e0 = s.mass_energy(q)
    if warmup > 0:
        s.step_relaxation(q, dt, warmup)
        s.step(q_plain, dt, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_end = s.step_relaxation(q, dt, steps, warmup * dt)
    sec = time.perf_counter() - t0
    s.step(q_plain, dt, steps)
    _, er = s.mass_energy(q)
    _, ec = s.mass_energy(q_plain)
    cells = grid.nx * grid.ny
    res = {"value": cells * 4 * steps / sec, "ms_per_step": sec / steps * 1e3, "dt": dt,
           "mean_gamma": (t_end - warmup * dt) / (steps * dt),
           "energy_drift_rel": (er - e0) / abs(e0), "classical_rk4_energy_drift_rel": (ec - e0) / abs(e0)}
    log(f"[relaxation] {res['value']:.4e} cell-stage/s  {res['ms_per_step']:.3f} ms/step  "
        f"dE/E {res['energy_drift_rel']:.2e} (classical {res['classical_rk4_energy_drift_rel']:.2e})")
    s.close()
    return res


def run_totals(problem, steps, warmup, tile_y):
    """RK4 steps with mass and energy recorded after every step (the step
    kernel's totals epilogue), against the plain step and against a separate
    totals pass after every step, on the main workload."""
    import torch
    from paper_2601_02540_amd.binding import Solver
    grid = problem.grid
    s = Solver(grid, torch.float64)
    if tile_y is not None:
        s.set_tile_y(tile_y)
    b = torch.from_numpy(problem.b).cuda()
    q = torch.from_numpy(problem.q0).cuda()
    s.set_bathymetry(b)
    s.init_aux(q)
    dt = s.cfl_dt(q, 0.5)
    _, e0 = s.mass_energy(q)
    s.step_totals(q, dt, warmup)
    s.step(q, dt, warmup)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(s.stream)
    series = s.step_totals(q, dt, steps)
    ev[1].record(s.stream)
    s.step(q, dt, steps)
    ev[2].record(s.stream)
    ev[2].synchronize()
    t_series = ev[0].elapsed_time(ev[1]) / steps
    t_plain = ev[1].elapsed_time(ev[2]) / steps
    # a separate totals call (one pass over the state, synchronizing)
    n_sep = 20
    t0 = time.perf_counter()
    for _ in range(n_sep):
        s.mass_energy(q)
    t_call = (time.perf_counter() - t0) / n_sep * 1e3
    e = series[:, 1].cpu()
    res = {"ms_per_step_recorded": t_series, "ms_per_step_plain": t_plain, "ms_totals_call": t_call,
           "energy_drift_rel_over_series": float((e[-1] - e[0]) / abs(e0)), "steps": steps}
    log(f"[totals] {t_series:.3f} ms/step with mass and energy recorded every step (plain step {t_plain:.3f}, "
        f"plus a separate totals call {t_call:.3f})")
    s.close()
    return res


def run_long_drift(problem, nsteps=1000):
    """The 4096^2 workload's whole 1000-step run in FP64 and in FP32 storage,
    mass and energy recorded after every step by the step kernel: relative
    drifts after 100, 500 and 1000 steps and the largest along the run."""
    import torch
    from paper_2601_02540_amd.binding import Solver
    out = {}
    for dtype, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        s = Solver(problem.grid, dtype)
        b = torch.from_numpy(problem.b).to(dtype).cuda()
        q = torch.from_numpy(problem.q0).to(dtype).cuda()
        s.set_bathymetry(b)
        s.init_aux(q)
        dt = s.cfl_dt(q, 0.5)
        m0, e0 = s.mass_energy(q)
        series = s.step_totals(q, dt, nsteps).cpu().numpy()
        dm = (series[:, 0] - m0) / abs(m0)
        de = (series[:, 1] - e0) / abs(e0)
        out[name] = {"steps": nsteps, "dt": dt,
                     "energy_drift_rel": {str(n): float(de[n - 1]) for n in (100, 500, nsteps)},
                     "mass_drift_rel": {str(n): float(dm[n - 1]) for n in (100, 500, nsteps)},
                     "max_abs_energy_drift_rel": float(abs(de).max()), "max_abs_mass_drift_rel": float(abs(dm).max())}
        log(f"[long run {name}] {nsteps} steps: energy drift {de[-1]:.3e} (max {abs(de).max():.3e}), "
            f"mass drift {dm[-1]:.3e}")
        s.close()
        del q, b
        torch.cuda.empty_cache()
    return out


def run_adaptive(nx, t_end, label, rtol=1e-6, atol=1e-6):
    """The adaptive five-stage FSAL pair at the paper's tolerances on the paper's
    Gaussian-obstacle setup (nx x nx/2, spacing 40/nx), from t = 0 to t_end,
    beside classical RK4 at the fixed CFL-0.5 step over the same interval.
    Right-hand-side evaluations: 5 per attempt (the FSAL stage is the next
    attempt's first), 4 per RK4 step."""
    import numpy as np
    import torch
    from paper_2601_02540_amd import workloads as W
    from paper_2601_02540_amd.binding import Solver
    p = W.gaussian_obstacle(nx)
    g = p.grid
    s = Solver(g, torch.float64)
    b = torch.from_numpy(p.b).cuda()
    q0 = torch.from_numpy(p.q0).cuda()
    s.set_bathymetry(b)
    s.init_aux(q0)
    dt_cfl = s.cfl_dt(q0, 0.5)
    m0, e0 = s.mass_energy(q0)
    q = q0.clone()
    s.step_adaptive(q, 0.0, 4 * dt_cfl, dt_cfl, rtol, atol)  # warm-up (buffers, graph)
    q.copy_(q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = s.step_adaptive(q, 0.0, t_end, dt_cfl, rtol, atol)
    wall = time.perf_counter() - t0
    m1, e1 = s.mass_energy(q)
    # the same run with one role kernel per evaluation (the four-stage path)
    s.set_step_path("stages")
    qs = q0.clone()
    s.step_adaptive(qs, 0.0, 4 * dt_cfl, dt_cfl, rtol, atol)
    qs.copy_(q0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res_roles = s.step_adaptive(qs, 0.0, t_end, dt_cfl, rtol, atol)
    wall_roles = time.perf_counter() - t2
    same_bits = bool(torch.equal(qs, q)) and res_roles == res
    s.set_step_path("fused")
    del qs
    # fixed-step RK4 over the same interval
    n_rk4 = math.ceil(t_end / dt_cfl)
    qr = q0.clone()
    s.prepare_step(qr, t_end / n_rk4, n_rk4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.step(qr, t_end / n_rk4, n_rk4)
    torch.cuda.synchronize()
    wall_rk4 = time.perf_counter() - t1
    _, er = s.mass_energy(qr)
    cells = g.nx * g.ny
    diff = float(torch.max(torch.abs(q[0] - qr[0])))
    out = {"grid": [g.nx, g.ny], "t_end": t_end, "rtol": rtol, "atol": atol, "wall_s": wall,
           "accepted": res["accepted"], "rejected": res["rejected"],
           "mean_step": t_end / res["accepted"], "cfl_step": dt_cfl,
           "ms_per_attempt": wall / res["attempts"] * 1e3,
           "rhs_evals_per_s": cells * 5 * res["attempts"] / wall,
           "role_kernels": {"wall_s": wall_roles, "ms_per_attempt": wall_roles / res_roles["attempts"] * 1e3,
                            "same_bits": same_bits},
           "mass_drift_rel": (m1 - m0) / abs(m0), "energy_drift_rel": (e1 - e0) / abs(e0),
           "rk4_fixed": {"steps": n_rk4, "wall_s": wall_rk4, "rhs_evals_per_s": cells * 4 * n_rk4 / wall_rk4,
                         "energy_drift_rel": (er - e0) / abs(e0)},
           "max_abs_h_diff_vs_rk4": diff}
    log(f"[{label}] {res['accepted']} accepted / {res['rejected']} rejected steps to t = {t_end} "
        f"(mean step {out['mean_step']:.3e}, CFL step {dt_cfl:.3e}) in {wall:.3f} s; "
        f"RK4 at the CFL step: {n_rk4} steps in {wall_rk4:.3f} s; role kernels: {wall_roles:.3f} s "
        f"(same bits: {same_bits})")
    # The same run in FP32 storage and arithmetic (error norm and controller in FP64 on the device): the
    # paper ran everything in FP64 after adaptive stepping misbehaved in FP32 in its implementation.
    qh = q.double().cpu()
    s.close()
    del q, qr, q0
    torch.cuda.empty_cache()
    s32 = Solver(g, torch.float32)
    q32 = torch.from_numpy(p.q0).float().cuda()
    s32.set_bathymetry(torch.from_numpy(p.b).float().cuda())
    s32.init_aux(q32)
    dt32 = s32.cfl_dt(q32, 0.5)
    q32_0 = q32.clone()
    s32.step_adaptive(q32, 0.0, 4 * dt32, dt32, rtol, atol)
    q32.copy_(q32_0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    res32 = s32.step_adaptive(q32, 0.0, t_end, dt32, rtol, atol)
    wall32 = time.perf_counter() - t3
    out["fp32"] = {"accepted": res32["accepted"], "rejected": res32["rejected"], "t": res32["t"],
                   "mean_step": t_end / max(res32["accepted"], 1), "wall_s": wall32,
                   "ms_per_attempt": wall32 / res32["attempts"] * 1e3, "last_err": res32["last_err"],
                   "max_abs_h_diff_vs_fp64": float(torch.max(torch.abs(q32[0].double().cpu() - qh[0])))}
    log(f"[{label} fp32] {res32['accepted']} accepted / {res32['rejected']} rejected steps in {wall32:.3f} s; "
        f"max |h - h_fp64| {out['fp32']['max_abs_h_diff_vs_fp64']:.2e}")
    s32.close()
    torch.cuda.empty_cache()
    return out


def torch_f64():
    import torch
    return torch.float64


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_child(spec):
    """Child-process leg (bench.py --oracle-child JSON): the FP64 oracle on the
    benchmark workload.  For each boundary type in spec["bcs"]: the oracle's own
    initialization and CFL step, totals at step 0 and after spec["drift_steps"]
    steps of its threaded build (timed: the all-core baseline), and on the first
    boundary type also spec["serial_steps"] steps of the serial build (timed:
    the single-thread baseline).  Prints one JSON line."""
    import oracle
    from paper_2601_02540_amd import workloads as W
    out = {"threads": oracle.threads_available(), "bcs": {}}
    for k, name in enumerate(spec["bcs"]):
        p = W.random_phase_large(spec["n"], W.PERIODIC if name == "periodic" else W.REFLECTING, seed=3)
        g = p.grid
        q = oracle.init_aux(g, p.q0, p.b)
        dt = oracle.cfl_dt(g, q, 0.5)
        m0, e0 = oracle.mass_energy(g, q, p.b)
        entry = {"dt": dt, "mass0": m0, "energy0": e0, "cells": g.nx * g.ny}
        if k == 0 and spec["serial_steps"] > 0:
            t0 = time.perf_counter()
            oracle.rk4(g, q, p.b, dt, spec["serial_steps"])
            entry["serial_s"] = time.perf_counter() - t0
            entry["serial_steps"] = spec["serial_steps"]
        m = spec["drift_steps"]
        with oracle.threaded():
            t0 = time.perf_counter()
            qm = oracle.rk4(g, q, p.b, dt, m)
            entry["threaded_s"] = time.perf_counter() - t0
        entry["drift_steps"] = m
        entry["mass"], entry["energy"] = oracle.mass_energy(g, qm, p.b)
        out["bcs"][name] = entry
    # smaller runs: the oracle's own totals after the same number of steps
    out["extra"] = {}
    for name, steps in spec.get("extra", {}).items():
        p = extra_problem(name)
        g = p.grid
        q = oracle.init_aux(g, p.q0, p.b)
        dt = oracle.cfl_dt(g, q, 0.5)
        m0, e0 = oracle.mass_energy(g, q, p.b)
        with oracle.threaded():
            qm = oracle.rk4(g, q, p.b, dt, steps)
        m1, e1 = oracle.mass_energy(g, qm, p.b)
        out["extra"][name] = {"drift_steps": steps, "mass0": m0, "energy0": e0, "mass": m1, "energy": e1}
    print(json.dumps(out), flush=True)


def extra_problem(name):
    """The seeded workloads of the smaller bench runs, by name (each side builds its own)."""
    from paper_2601_02540_amd import workloads as W
    if name == "gaussian_bump_64":
        return W.gaussian_bump_periodic(64, seed=1)
    if name == "soliton_512":
        return W.soliton_over_bathymetry(512, seed=2)
    if name.startswith("ensemble_"):
        return W.ensemble(256, seed=4)[int(name.split("_")[1])]
    raise ValueError(name)


def run_oracle_child(n, bcs, drift_steps, serial_steps, extra=None):
    """Runs oracle_child in a fresh process.  glibc would return every freed
    plane to the system and fault it in again, page by page and serially, on
    the next call; the child keeps freed memory in its heap instead (malloc
    thresholds set in its environment), which only changes where the oracle's
    buffers come from."""
    import subprocess
    env = dict(os.environ, MALLOC_MMAP_THRESHOLD_=str(1 << 40), MALLOC_TRIM_THRESHOLD_=str(1 << 42))
    spec = {"n": n, "bcs": bcs, "drift_steps": drift_steps, "serial_steps": serial_steps, "extra": extra or {}}
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-child", json.dumps(spec)],
                       env=env, capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(orc):
    """The oracle as it stands, timed on the host: the threaded build over all
    usable cores (value) and the serial build on one (single_thread)."""
    first = next(iter(orc["bcs"].values()))
    cells = first["cells"]
    thr = cells * 4 * first["drift_steps"] / first["threaded_s"]
    res = {"value": thr, "unit": "cell-stage/s", "cores": orc["threads"], "kind": "oracle",
           "sample": f"{first['drift_steps']} RK4 steps of the same {int(math.isqrt(cells))}^2 FP64 workload "
                     f"({first['threaded_s']:.1f} s; C++ -O2 -ffp-contract=off, OpenMP build, "
                     f"{orc['threads']} threads)", **cpu_info()}
    if "serial_s" in first:
        res["single_thread"] = {"value": cells * 4 * first["serial_steps"] / first["serial_s"], "cores": 1,
                                "sample": f"{first['serial_steps']} RK4 steps, serial build "
                                          f"({first['serial_s']:.1f} s)"}
    return res


def vs_oracle(gpu_res, orc_entry, d=None):
    """Totals after the same number of steps from each side's own initialization
    of the workload: GPU (any storage type) against the FP64 oracle."""
    d = gpu_res.get("drift_series") if d is None else d
    if d is None or orc_entry is None or d["steps"] != orc_entry["drift_steps"]:
        return None
    return {"steps": d["steps"],
            "gpu_energy_drift_rel": (d["energy"] - d["energy0"]) / abs(d["energy0"]),
            "oracle_energy_drift_rel": (orc_entry["energy"] - orc_entry["energy0"]) / abs(orc_entry["energy0"]),
            "energy_diff_rel": (d["energy"] - orc_entry["energy"]) / abs(orc_entry["energy"]),
            "mass_diff_rel": (d["mass"] - orc_entry["mass"]) / abs(orc_entry["mass"]),
            "gpu_mass_drift_rel": (d["mass"] - d["mass0"]) / abs(d["mass0"]),
            "oracle_mass_drift_rel": (orc_entry["mass"] - orc_entry["mass0"]) / abs(orc_entry["mass0"])}


def step_sources_unchanged():
    import hashlib
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_02540_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest() == STEP_SOURCES_SHA256


def roofline(path, res, cells, esize=8):
    """Roofline entry of the main run's dominant kernel, against HBM: the
    algorithmic bytes of one launch (the method's own values per node, see
    PATHS) over the mean launch duration inside the timed region.  For the
    step kernel the FP64 arithmetic rate (FLOPS_PER_NODE_STEP per node) is
    reported beside it."""
    values, launches = PATHS[path]
    traffic = None
    if path == "fused" and esize == 8 and cells == 4096 * 4096 and res["tile_y"] in (None, 24) and \
            step_sources_unchanged():
        traffic = STEP_TRAFFIC_BYTES_PER_NODE * cells
    out = dict(bound="hbm", achieved=res["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=res["frac"],
               traffic=traffic, kernel=KERNELS[path], traffic_unit="bytes per launch",
               launch_us=res["stage_launch_us"],
               algorithmic_bytes_per_launch_per_node=values / launches * esize,
               algorithmic_bytes_per_step_per_node=values * esize)
    if path == "fused":
        tflops = FLOPS_PER_NODE_STEP * cells / (res["stage_launch_us"] * 1e-6) / 1e12
        out.update(fp64_achieved_TFLOPs=tflops, fp64_peak_TFLOPs=FP64_VECTOR_PEAK_TFLOPS,
                   fp64_frac=tflops / FP64_VECTOR_PEAK_TFLOPS, flops_per_node_step=FLOPS_PER_NODE_STEP)
    return out


def calib_copy(nbytes):
    """A plain device copy of known size, for scaling rocprof FETCH_SIZE/WRITE_SIZE."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[calib] copied {nbytes} bytes x3")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=4096, help="grid nodes per axis")
    ap.add_argument("--no-variants", action="store_true", help="skip the reflecting and FP32 repeats")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path", choices=sorted(PATHS), default="fused", help="step path of the main run")
    ap.add_argument("--tile-y", type=int, choices=(8, 16, 24), default=None,
                    help="tile height (default: the library's defaults; 24 = 32 x 24 step tiles)")
    ap.add_argument("--variants", default="all",
                    help="comma list of extra runs: f32,reflecting,ensemble,small,adjoint,paths,paper,relaxation,"
                         "totals,adaptive,longdrift (default all)")
    ap.add_argument("--ensemble-steps", type=int, default=100)
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--calib-copy", type=int, default=0, help="also copy this many bytes (counter calibration)")
    ap.add_argument("--long-dam-break", action="store_true",
                    help="also run the 10^8-node cylindrical dam break to t = 300 (several minutes)")
    ap.add_argument("--repeats", type=int, default=5, help="timed repeats of --steps steps (median reported)")
    ap.add_argument("--drift-steps", type=int, default=10,
                    help="steps over which the 4096^2 runs' totals are compared with the FP64 oracle's (0: skip)")
    ap.add_argument("--oracle-serial-steps", type=int, default=2,
                    help="steps of the serial oracle in the single-thread CPU baseline")
    ap.add_argument("--oracle-child", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.oracle_child is not None:
        oracle_child(json.loads(args.oracle_child))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the kernels are measured on one GPU's share); "
                                   "--gpus must be 1",
                          "requested_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2601_02540_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no ROCm GPU visible"}), flush=True)
        sys.exit(1)

    if args.calib_copy:
        calib_copy(args.calib_copy)

    n = args.n
    log(f"[bench] generating {n}x{n} workload")
    prob = W.random_phase_large(n, W.PERIODIC, seed=3)
    P, T = args.path, args.tile_y
    R, DS = max(args.repeats, 1), max(args.drift_steps, 0)
    main_res = run_gpu(prob, torch.float64, args.steps, args.warmup, "periodic f64", P, T, R, DS)

    variants = {}
    chosen = set() if args.no_variants else (ALL_VARIANTS if args.variants == "all" else set(args.variants.split(",")))
    unknown = chosen - ALL_VARIANTS
    if unknown:
        raise SystemExit(f"unknown variants: {sorted(unknown)}; choose from {sorted(ALL_VARIANTS)}")
    if "f32" in chosen:
        variants["periodic_f32"] = run_gpu(prob, torch.float32, args.steps, args.warmup, "periodic f32", P, T, R, DS,
                                           SETTLE_STEPS)
        variants["periodic_f32"]["energy_diff_vs_f64_rel"] = (
            (variants["periodic_f32"]["energy_final"] - main_res["energy_final"]) / abs(main_res["energy_final"]))
    if "reflecting" in chosen:
        probr = W.random_phase_large(n, W.REFLECTING, seed=3)
        variants["reflecting_f64"] = run_gpu(probr, torch.float64, args.steps, args.warmup, "reflecting f64", P, T,
                                             R, DS, SETTLE_STEPS)
        variants["reflecting_f32"] = run_gpu(probr, torch.float32, args.steps, args.warmup, "reflecting f32", P, T,
                                             R, DS, SETTLE_STEPS)
    if "ensemble" in chosen:
        variants["ensemble_256_f32"] = run_ensemble(256, args.ensemble_steps, 4, torch.float32, "ensemble f32",
                                                    "pairs" if P == "pairs" else "fused")
    if "small" in chosen:
        small = W.gaussian_bump_periodic(64, seed=1)
        variants["gaussian_bump_64_f64"] = run_gpu(small, torch.float64, 200, 8, "gaussian bump 64 f64", P, T, R,
                                                   200 if DS > 0 else 0, SETTLE_STEPS)
        sol = W.soliton_over_bathymetry(512, seed=2)
        variants["soliton_512_reflecting_f64"] = run_gpu(sol, torch.float64, 500, 8, "soliton 512 f64", P, T, R,
                                                         50 if DS > 0 else 0, SETTLE_STEPS)
    if "adjoint" in chosen:
        variants["adjoint_gauges_1024_f64"] = run_adjoint(1024, args.adjoint_steps, "adjoint 1024 f64")
    if "relaxation" in chosen:
        variants["relaxation_f64"] = run_relaxation(prob, min(args.steps, 200), 8, P, T)
    if "totals" in chosen:
        variants["recorded_totals_f64"] = run_totals(prob, min(args.steps, 200), 8, T)
    if "adaptive" in chosen:
        variants["adaptive_fsal_gaussian_obstacle_1600x800"] = run_adaptive(1600, 0.5, "adaptive pair 1600x800")
    if "longdrift" in chosen and n == 4096:
        variants["long_run_1000_steps_4096"] = run_long_drift(prob, 1000)
    if "paper" in chosen:
        variants["paper_setups"] = run_paper_setups(P, T)
    if args.long_dam_break:
        variants["cylindrical_dam_break_to_t300"] = run_long_dam_break(P, T)
    if "paths" in chosen:
        for other in sorted(PATHS):
            if other != P:
                variants[f"periodic_f64_{other}"] = run_gpu(prob, torch.float64, args.steps, args.warmup,
                                                            f"periodic f64 {other}", other, T, R, 0, SETTLE_STEPS)

    cpu = None
    if not args.no_cpu_baseline or DS > 0:
        bcs = ["periodic"] + (["reflecting"] if "reflecting_f64" in variants and DS > 0 else [])
        log(f"[bench] FP64 oracle on the same workload ({', '.join(bcs)}): {DS} threaded steps, "
            f"{0 if args.no_cpu_baseline else args.oracle_serial_steps} serial")
        extra = {}
        if DS > 0:
            for key, name in (("gaussian_bump_64_f64", "gaussian_bump_64"), ("soliton_512_reflecting_f64", "soliton_512")):
                if key in variants and "drift_series" in variants[key]:
                    extra[name] = variants[key]["drift_series"]["steps"]
            for name, d in variants.get("ensemble_256_f32", {}).get("drift_instances", {}).items():
                extra[name] = d["steps"]
        orc = run_oracle_child(n, bcs, max(DS, 1), 0 if args.no_cpu_baseline else args.oracle_serial_steps, extra)
        if not args.no_cpu_baseline:
            cpu = cpu_baseline(orc)
            log(f"[bench] cpu {cpu['value']:.3e} cell-stage/s on {cpu['cores']} threads")
        for name, res in [("periodic", main_res)] + [(k.split("_")[0], v) for k, v in variants.items()
                                                     if k in ("periodic_f32", "reflecting_f64", "reflecting_f32")]:
            res["energy_vs_oracle"] = vs_oracle(res, orc["bcs"].get(name))
        for key, name in (("gaussian_bump_64_f64", "gaussian_bump_64"), ("soliton_512_reflecting_f64", "soliton_512")):
            if key in variants:
                variants[key]["energy_vs_oracle"] = vs_oracle(variants[key], orc.get("extra", {}).get(name))
        ens = variants.get("ensemble_256_f32")
        if ens is not None:
            ens["energy_vs_oracle"] = {name: vs_oracle(ens, orc.get("extra", {}).get(name), dict(d, steps=d["steps"]))
                                       for name, d in ens.get("drift_instances", {}).items()}

    cells = n * n
    line = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"random-phase bathymetry, Gaussian bump, periodic [-50,50]^2, {n}x{n}, "
                               f"lambda=500, RK4 fixed dt (CFL 0.5)",
                   "nx": n, "ny": n, "cells": cells, "bc": "periodic", "lambda": 500.0, "g": 9.81,
                   "dt": main_res["dt"], "parallelism": "single GPU"},
        "roofline": roofline(P, main_res, cells),
        "repeats": R,
        "ms_per_step_repeats": main_res["ms_per_step_repeats"],
        "energy_vs_oracle": main_res.get("energy_vs_oracle"),
        "cpu_baseline": cpu,
        "energy_drift_rel": main_res["energy_drift_rel"],
        "energy_drift_rel_to_excess": main_res["energy_drift_rel_to_excess"],
        "mass_drift_rel": main_res["mass_drift_rel"],
        "kernel_ms": main_res["kernel_ms"],
        "variants": {k: {kk: vv for kk, vv in v.items() if kk not in ("energy_final", "drift_series")}
                     for k, v in variants.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
