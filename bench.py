#!/usr/bin/env python3
"""Throughput of the DPD step with phase-field no-slip walls on one MI355X.

One step = the whole hot path on one batch of synthetic particles: drift +
phase-field bounce-back + binning, the counting-sort cell list, and the
pairwise conservative + dissipative + random force with the velocity update
(all in the library's HIP kernels).  Inputs are resident in HBM before the
timed region; the timed region is exactly --steps steps between two stream
synchronisations.  Prints one JSON line on stdout; progress goes to stderr.

Default workload: porous medium (thresholded Gaussian random field,
correlation length 6, porosity 0.35) in a 168^3 periodic box at density 4,
phi on a 672^3 float32 grid, ~8.5M fluid + wall particles (the 128^3 box as
written holds ~3.7M after the solid is carved out).
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

HBM_PEAK_GBS = 8000.0
# Per-unit VALU work of the pair force (full-rate instruction slots per
# lane, a model): an interacting pair costs ~40 for the force, ~100 for
# Philox4x32-10 (its ten 32 x 32 -> 64-bit multiplies issue at a quarter of
# the full rate) and ~20 for Box-Muller; a candidate test ~10.  The unit is
# the Newton-3 pair (each fluid-fluid pair once, each fluid-wall pair once)
# and the half-shell candidate (each fluid-fluid candidate once, each
# fluid-wall candidate once).
OPS_PER_PAIR = 160
OPS_PER_CANDIDATE = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads
    if name == "porous168":
        return workloads.porous_system(Lbox=168.0, name="porous_grf_168", device="cuda")
    if name == "porous128":
        return workloads.porous_system(Lbox=128.0, name="porous_grf_128", device="cuda")
    if name == "channel":
        return workloads.sinusoid_cylinder_system()
    if name == "slab":
        return workloads.slab_system()
    raise ValueError(name)


def algorithmic_counts(sim, system):
    """Interacting pairs from the library's own pair list, split into
    fluid-fluid (each counted once) and fluid-wall, and half-shell candidate
    pairs from the cell occupancy: each fluid-fluid candidate in the 27 cells
    around a fluid particle once, each fluid-wall candidate once."""
    import numpy as np
    import torch
    from paper_1807_09896_amd import binding
    total = binding.dpd_neighbor_pairs(sim.ctx, None, 0)
    buf = torch.empty((total, 2), dtype=torch.int32, device="cuda")
    got = binding.dpd_neighbor_pairs(sim.ctx, buf, total)
    assert got == total
    typ = np.empty_like(system.type)
    typ[system.gid] = system.type
    wall_of_gid = torch.from_numpy((typ != 0).astype(np.int8)).to("cuda")
    fw = int(wall_of_gid[buf[:, 1].long()].sum())
    del buf
    ff_directed = total - fw
    st = sim.state()
    cell = st["cell_of"].cpu().numpy()
    L = system.L
    rc = system.params["rc"]
    nc = [int(math.floor(x / rc)) for x in L]
    ncell = nc[0] * nc[1] * nc[2]
    shape = (nc[2], nc[1], nc[0])
    nf_c = np.bincount(cell[typ == 0], minlength=ncell).reshape(shape).astype(np.int64)
    nw_c = np.bincount(cell[typ != 0], minlength=ncell).reshape(shape).astype(np.int64)
    Sf = np.zeros_like(nf_c)
    Sw = np.zeros_like(nw_c)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                Sf += np.roll(nf_c, (dz, dy, dx), axis=(0, 1, 2))
                Sw += np.roll(nw_c, (dz, dy, dx), axis=(0, 1, 2))
    ff_cands = int((nf_c * (Sf - 1)).sum()) // 2
    fw_cands = int((nf_c * Sw).sum())
    return dict(pairs_ff=ff_directed // 2, pairs_fw=fw, pairs_directed=total,
                candidates_ff_half=ff_cands, candidates_fw=fw_cands,
                candidates_full=2 * ff_cands + fw_cands, cells=ncell)


def valu_peak(ms_target=20.0):
    """Issue rate of the vector ALU, measured: the library's calibration
    kernel runs 64 x iters v_fmac_f32 per lane on 16 wavefronts per SIMD
    (every SIMD of the chip busy); lane-op slots per second."""
    import torch
    from paper_1807_09896_amd import binding
    props = torch.cuda.get_device_properties(0)
    waves = props.multi_processor_count * 4 * 16
    out = torch.empty(waves * 64, dtype=torch.float32, device="cuda")
    binding.dpd_valu_probe(0, waves, 10, out)
    iters = 400
    best = 0.0
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        binding.dpd_valu_probe(0, waves, iters, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = max(best, waves * 64.0 * 64 * iters / (ms * 1e-3))
        if ms < ms_target:
            iters = int(iters * ms_target / max(ms, 1e-3))
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="porous168",
                    choices=["porous168", "porous128", "channel", "slab"])
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the launch shapes of the main run")
    ap.add_argument("--graph", action="store_true",
                    help="replay each step of the main run as a captured HIP graph")
    ap.add_argument("--timing-steps", type=int, default=20,
                    help="steps of the per-kernel HIP-event pass")
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps of the CPU baseline (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="steps of the 256-replica batch leg and of its sequential "
                         "comparison (0 skips the leg)")
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--walls-steps", type=int, default=200,
                    help="steps of the moving-wall leg (plane Couette channel); 0 skips it")
    ap.add_argument("--sph-steps", type=int, default=100,
                    help="steps of the attractive-repulsive force leg (the same workload "
                         "with the Eq. 22-24 force); 0 skips it")
    ap.add_argument("--phase-field-iters", type=int, default=200,
                    help="relaxation steps of the phase-field leg (Eq. 15 on the workload's "
                         "grid from its step function); 0 skips it")
    ap.add_argument("--stokes-steps", type=int, default=2000,
                    help="steps of the cylinder-array leg (16 replica cells of Sec. III.B "
                         "in one batch); 0 skips it")
    ap.add_argument("--adjoint-reps", type=int, default=3,
                    help="timed repetitions of the 200-step adjoint window (0 skips the leg)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy this many MiB with the library's plain copy "
                         "kernel (the reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1807_09896_amd as dpd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    system = make_workload(args.workload)
    log("workload %s: %d particles (%d fluid, %d wall), phi %s %s, generated in %.1fs"
        % (system.name, system.n, system.n_fluid, system.n_wall, system.phi.shape,
           system.phi.dtype, time.time() - t0))
    sim = dpd.Simulation(system, graph=args.graph)
    cnt0 = sim.counters()
    log("created:", cnt0)
    shape = None
    if args.autotune:
        shape, trials = sim.autotune(5)
        log("autotuned shape (particles/thread, force block) = %s; trial ms/step %s"
            % (shape, ["%.3f" % t for t in trials]))

    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    sec = tb - ta
    ms_per_step = sec * 1e3 / max(args.steps, 1)
    value = system.n * args.steps / sec
    log("timed %d steps: %.4f ms/step, %.4e particle-steps/s" % (args.steps, ms_per_step, value))

    # per-kernel HIP events on the library stream
    sim.kernel_times(1)
    sim.step(args.timing_steps)
    kt = sim.kernel_times(0)
    lk1 = sim.counters()
    for k, (ms, c) in kt.items():
        if c:
            log("  %-24s %9.4f ms/launch x %d" % (k, ms / c, c))
    f_ms, f_n = kt["pair_force"]
    # a step launches the pair force once per kernel kind that has work
    force_launches_per_step = max(1, round(f_n / max(args.timing_steps, 1)))
    force_ms = f_ms / max(args.timing_steps, 1)
    cnt = algorithmic_counts(sim, system)
    ncell = cnt["cells"]
    lookups = lk1["phi_lookups"]
    pairs_unique = cnt["pairs_ff"] + cnt["pairs_fw"]
    cands_half = cnt["candidates_ff_half"] + cnt["candidates_fw"]
    ops = pairs_unique * OPS_PER_PAIR + cands_half * OPS_PER_CANDIDATE
    valu = valu_peak()
    achieved_valu = ops / (force_ms * 1e-3)
    nf, nw = system.n_fluid, system.n_wall
    b_alg = nf * (72 + 16 + 28 + 12 + 1) + 16 * nw + 8 * ncell + (
        64 if system.phi.dtype == np.float64 else 32) * lookups
    # the step's duration from the same HIP-event pass: the sum of its
    # kernels' event-timed launches per step
    step_event_ms = sum(ms for ms, c in kt.values() if c) / max(args.timing_steps, 1)
    step_gbs = b_alg / (step_event_ms * 1e-3) / 1e9
    # the pair force's own algorithmic bytes: positions, predicted velocities
    # and gids of fluid and walls read once, the state written once in cell
    # order (r, v, f: 48 B per fluid particle), the merged cell runs read once
    force_bytes = nf * (32 + 48) + 32 * nw + 4 * (nf + nw) + 8 * ncell
    force_gbs = force_bytes / (force_ms * 1e-3) / 1e9
    log("pairs: %d fluid-fluid (each once), %d fluid-wall (%.2f per fluid particle); "
        "half-shell candidates %d; phi lookups/step %.0f; B_alg %.1f MB"
        % (cnt["pairs_ff"], cnt["pairs_fw"], pairs_unique / max(nf, 1), cands_half, lookups,
           b_alg / 1e6))
    log("step: %.1f GB/s of algorithmic traffic = %.4f of HBM peak; pair_force %.4f ms per step, "
        "%.3e VALU slots/s by the model = %.3f of the measured VALU issue rate %.3e/s"
        % (step_gbs, step_gbs / HBM_PEAK_GBS, force_ms, achieved_valu, achieved_valu / valu, valu))

    if args.copy_probe_mb > 0:
        from paper_1807_09896_amd import binding
        nbytes = args.copy_probe_mb << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        binding.dpd_copy_probe(b, a, nbytes)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read and written by k_copy16" % nbytes)
        del a, b

    prof_dir = os.path.join(ROOT, "profiles")
    traffic = force_traffic = None
    tfile = os.path.join(prof_dir, "step_%s_traffic.json" % args.workload)
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_step")
            force_traffic = tr.get("pair_force_bytes_per_step")

    pfield = None
    if args.phase_field_iters > 0:
        pfield = phase_field_leg(dpd, system, args.phase_field_iters)

    sph = None
    if args.sph_steps > 0:
        sim.close()
        sph = sph_leg(dpd, system, args.sph_steps, args.timing_steps, force_ms, ms_per_step)

    batch = None
    if args.batch_steps > 0:
        sim.close()
        batch = batch_leg(dpd, args.replicas, args.batch_steps)

    adjoint = None
    if args.adjoint_reps > 0:
        sim.close()
        adjoint = adjoint_leg(dpd, args.adjoint_reps)

    walls = None
    if args.walls_steps > 0:
        walls = walls_leg(dpd, args.walls_steps)

    stokes = None
    if args.stokes_steps > 0:
        stokes = stokes_leg(dpd, args.stokes_steps)

    cpu = None
    if args.cpu_steps > 0:
        import oracle
        oracle.build_oracle(force=False)
        log("cpu baseline: oracle on %d threads, %d steps of the same workload"
            % (oracle.num_threads(), args.cpu_steps))
        o = oracle.Oracle(system)
        tc = time.perf_counter()
        o.step(args.cpu_steps)
        tcs = time.perf_counter() - tc
        cpu = {"value": system.n * args.cpu_steps / tcs, "unit": "particle-steps/s",
               "cores": oracle.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
               "sample": "%d full steps of the same %d-particle workload (FP64 C oracle, "
                         "OpenMP over particles), %.1f s" % (args.cpu_steps, system.n, tcs)}
        log("cpu baseline %.4e particle-steps/s in %.1fs" % (cpu["value"], tcs))

    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": system.name, "particles": system.n, "fluid": nf, "wall": nw,
                   "box": [float(x) for x in system.L], "density": 4.0 if "porous" in system.name else 3.0,
                   "phi_grid": list(system.phi.shape), "phi_dtype": str(system.phi.dtype),
                   "dt": system.params["dt"], "graph": bool(args.graph),
                   "launch_shape": list(shape) if shape else None,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "step (integrate + cell list + pair_force)",
                     "achieved": step_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": step_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": b_alg, "avg_step_ms": step_event_ms,
                     "avg_step_ms_from": "HIP events on the library stream, sum of the "
                                         "step's kernels over %d steps" % args.timing_steps,
                     "traffic_GBs": (traffic / (step_event_ms * 1e-3) / 1e9
                                     if traffic else None)},
        "pair_force": {"avg_ms_per_step": force_ms, "launches_per_step": force_launches_per_step,
                       "pairs_ff": cnt["pairs_ff"], "pairs_fw": cnt["pairs_fw"],
                       "candidates_ff_half": cnt["candidates_ff_half"],
                       "candidates_fw": cnt["candidates_fw"],
                       "valu": {"bound": "valu", "achieved": achieved_valu, "peak": valu,
                                "unit": "VALU slots/s", "frac": achieved_valu / valu,
                                "model_ops_per_step": ops,
                                "peak_from": "dpd_valu_probe v_fmac_f32, measured in this run"},
                       "hbm": {"algorithmic_bytes": force_bytes, "achieved_GBs": force_gbs,
                               "frac": force_gbs / HBM_PEAK_GBS, "traffic": force_traffic}},
        "cpu_baseline": cpu,
        "batch": batch,
        "adjoint": adjoint,
        "moving_walls": walls,
        "sph_force": sph,
        "phase_field": pfield,
        "cylinder_array": stokes,
    }
    print(json.dumps(out), flush=True)
    sim.close()


def phase_field_leg(dpd, system, iters):
    """Phase-field relaxation (Sec. II.B, Eq. 15) of the workload's grid from
    its step function (-1 solid, +1 fluid) with sqrt(2) eps = 0.5, the
    interface width of the workload's tanh field, and dtau at half the
    explicit bound.  One launch per pseudo-time step; the launches are timed
    with HIP events on the stream they run on.  Algorithmic traffic: one
    read and one write of every node per step."""
    import numpy as np
    import torch
    t0 = time.time()
    phi = torch.from_numpy(system.phi).to("cuda")
    phi = torch.where(phi > 0, 1.0, -1.0).to(phi.dtype).contiguous()
    work = torch.empty(phi.numel() + 1, dtype=phi.dtype, device="cuda")
    h = [float(x) for x in system.h]
    eps = 0.5 / math.sqrt(2.0)
    dtau = 0.5 / (2.0 * sum((eps / x) ** 2 for x in h))
    es = phi.element_size()
    dpd.dpd_phi_relax(phi, work, h, eps, dtau, 2, residual=False)
    torch.cuda.synchronize()
    iters -= iters % 2
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    dpd.dpd_phi_relax(phi, work, h, eps, dtau, iters, residual=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    res = dpd.dpd_phi_relax(phi, work, h, eps, dtau, 2, residual=True)
    nodes = phi.numel()
    gbs = 2 * es * nodes / (ms * 1e-3) / 1e9
    frac_interface = float((phi.abs() < 0.9).float().mean())
    del phi, work
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "phi_relax_porous168_traffic.json")
    if os.path.exists(tfile) and system.name == "porous_grf_168":
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("kernel_source_hash") == kernel_source_hash(("phase_field.hip",)):
            traffic = tr.get("bytes_per_launch")
    log("phase-field leg: %d nodes (%s), %.4f ms per step, %.1f GB/s (%.3f of HBM peak), "
        "residual after %d steps %.3e" % (nodes, "f%d" % (8 * es), ms, gbs, gbs / HBM_PEAK_GBS,
                                          iters + 4, res))
    return {"grid": list(system.phi.shape[::-1]), "dtype": "f%d" % (8 * es), "steps": iters,
            "eps": eps, "dtau": dtau, "ms_per_step": ms,
            "roofline": {"bound": "hbm", "kernel": "k_phi_relax", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "traffic": traffic, "bytes_per_launch": 2 * es * nodes,
                         "avg_launch_ms": ms},
            "residual_after": res, "pseudo_time": (iters + 4) * dtau,
            "interface_fraction": frac_interface, "seconds": time.time() - t0}


def stokes_leg(dpd, steps, replicas=16, solid_fraction=0.1):
    """Stokes flow through a square array of cylinders (Sec. III.B): 16
    replica cells (28 x 28 x 4, one cylinder of solid fraction 0.1 each,
    density 4, kBT = 0.1, gamma = 45, g = 0.001) stepped as one batch with
    graph replay."""
    import torch
    import workloads
    cells = [workloads.cylinder_array_system(solid_fraction=solid_fraction, seed=300 + k,
                                             params=workloads.stokes_params(g=0.001, seed=400 + k))
             for k in range(replicas)]
    n = sum(c.n for c in cells)
    sim = dpd.Simulation(cells, graph=True)
    sim.step(50)
    sim.sync()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    sim.close()
    log("cylinder-array leg: %d replicas, %d particles, %.4f ms/step, %.4e particle-steps/s"
        % (replicas, n, dt * 1e3 / steps, n * steps / dt))
    return {"workload": "cylinder_array", "replicas": replicas, "solid_fraction": solid_fraction,
            "particles": n, "steps": steps, "ms_per_step": dt * 1e3 / steps,
            "value": n * steps / dt, "unit": "particle-steps/s"}


def sph_leg(dpd, system, steps, timing_steps, force_ms, ms_per_step):
    """The attractive-repulsive conservative force of Eq. 22-24 on the same
    workload (Sec. IV's fluid: kBT = 0.5, the paper's strengths and ranges,
    fluid-solid strengths twice the fluid-fluid ones, dt = 0.005): whole
    step and pair-force launch against the linear force's."""
    import dataclasses
    import torch
    import workloads
    p = dict(system.params, sph=workloads.sph_force(), kBT=0.5, dt=0.005)
    s = dataclasses.replace(system, params=p)
    sim = dpd.Simulation(s)
    sim.step(20)
    sim.sync()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    sim.kernel_times(1)
    sim.step(timing_steps)
    kt = sim.kernel_times(0)
    c = sim.counters()
    sim.close()
    f_ms, f_n = kt["pair_force"]
    f_ms /= max(f_n, 1)
    log("sph leg: %.4f ms/step, %.4e particle-steps/s, pair_force %.4f ms/launch (linear force %.4f)"
        % (dt * 1e3 / steps, s.n * steps / dt, f_ms, force_ms))
    return {"workload": system.name, "particles": s.n, "steps": steps,
            "ms_per_step": dt * 1e3 / steps, "value": s.n * steps / dt,
            "unit": "particle-steps/s", "pair_force_ms": f_ms,
            "pair_force_ms_linear": force_ms, "step_ms_linear": ms_per_step,
            "unstable": c["unstable"]}


def batch_leg(dpd, replicas, steps):
    """Independent replica boxes of uneven size and geometry: one batch
    context (one launch per kernel for all boxes, autotuned launch shapes,
    step replayed as a HIP graph) against the same boxes as separate
    graph-replayed plain contexts stepped back to back."""
    import torch
    import workloads
    t0 = time.time()
    boxes = workloads.replica_systems(count=replicas)
    n_tot = sum(b.n for b in boxes)
    log("batch leg: %d replicas, %d particles (%d..%d per box), generated in %.1fs"
        % (replicas, n_tot, min(b.n for b in boxes), max(b.n for b in boxes), time.time() - t0))
    bsim = dpd.Simulation(boxes, graph=True)
    shape, trials = bsim.autotune(5)
    log("autotuned shape (particles/thread, force block) = %s; trial ms/step %s"
        % (shape, ["%.3f" % t for t in trials]))
    bsim.step(10)
    bsim.sync()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    bsim.step(steps)
    bsim.sync()
    torch.cuda.synchronize()
    tb_ = time.perf_counter() - ta
    bsim.kernel_times(1)
    bsim.step(5)
    kt = bsim.kernel_times(0)
    bsim.close()
    # the same batch as one persistent launch per step (dpd_use_persistent)
    psim = dpd.Simulation(boxes, graph=True)
    psim.use_persistent(True)
    psim.step(3)
    psim.sync()
    psteps = max(5, steps // 5)
    ta = time.perf_counter()
    psim.step(psteps)
    psim.sync()
    tp = (time.perf_counter() - ta) * 1e3 / psteps
    psim.close()
    log("persistent launch per step: %.4f ms/step" % tp)
    batched = n_tot * steps / tb_
    log("batched: %.4f ms/step, %.4e particle-steps/s" % (tb_ * 1e3 / steps, batched))
    sims = [dpd.Simulation(b, graph=True) for b in boxes]
    for s in sims:
        s.step(2)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for s in sims:
        s.step(steps)
    for s in sims:
        s.sync()
    torch.cuda.synchronize()
    ts = time.perf_counter() - ta
    for s in sims:
        s.close()
    seq = n_tot * steps / ts
    log("sequential plain contexts: %.4f ms per step of all boxes, %.4e particle-steps/s"
        % (ts * 1e3 / steps, seq))
    return {"replicas": replicas, "particles": n_tot, "steps": steps,
            "value": batched, "unit": "particle-steps/s", "ms_per_step": tb_ * 1e3 / steps,
            "sequential_value": seq, "sequential_ms_per_step": ts * 1e3 / steps,
            "speedup_vs_sequential": batched / seq, "shape": list(shape),
            "trial_ms_per_step": trials, "graph": True, "persistent_ms_per_step": tp,
            "kernel_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt.items() if v[1]}}


def walls_leg(dpd, steps, L=(192.0, 192.0, 10.0)):
    """Moving walls and specular reflection: a plane Couette channel (fluid
    1.5 < z < 8.5 at density 3, the plate above sliding at U = 1), stepped
    with resting plates, with the sliding plate (bounce-back: the walls
    translate and are re-sorted every step, reflections look up the plate's
    velocity) and with the sliding plate and specular reflection."""
    import torch
    import workloads
    import dataclasses
    t0 = time.time()
    base = workloads.couette_system(L=L, U=1.0, seed=80)
    walls = base.type != 0
    res = {}
    for name, U, spec in (("resting", 0.0, False), ("sliding", 1.0, False),
                          ("sliding_specular", 1.0, True)):
        vel = base.vel.copy()
        if U == 0.0:
            vel[walls] = 0.0
        s = dataclasses.replace(base, vel=vel, params=dict(base.params, specular=spec))
        sim = dpd.Simulation(s, graph=True)
        sim.step(20)
        sim.sync()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        c = sim.counters()
        sim.close()
        res[name] = {"ms_per_step": dt * 1e3 / steps, "value": s.n * steps / dt,
                     "unit": "particle-steps/s", "bounces_per_step": c["bounce"] / (steps + 20)}
        log("walls leg %-16s %d particles: %.4f ms/step, %.4e particle-steps/s" %
            (name, s.n, dt * 1e3 / steps, s.n * steps / dt))
    return {"workload": "couette_channel", "box": list(L), "particles": s.n,
            "fluid": int((s.type == 0).sum()), "steps": steps, **res,
            "generated_in_s": time.time() - t0}


def adjoint_leg(dpd, reps, steps=200, ckpt=20, nbins=40):
    """The differentiation workload: 20^3 slit with sinusoidal walls, a
    200-step window with a checkpoint every 20 steps, 40 bins along z.
    Times the recorded forward window and the backward sweep (segment
    recompute included) of the same window."""
    import numpy as np
    import torch
    import workloads
    from paper_1807_09896_amd import binding
    from paper_1807_09896_amd.adjoint import Window
    s = workloads.sinusoid_slit_system()
    sim = dpd.Simulation(s, graph=True)
    shape, _ = sim.autotune(5)
    win = Window(sim, steps=steps, ckpt=ckpt, axis=2, nbins=nbins)
    prof = win.run()
    dldp = (2.0 * (prof - 0.5 * prof) / nbins).contiguous()
    win.backward(dldp)
    tf, tb = [], []
    for _ in range(reps):
        binding.dpd_set_state(sim.ctx, win.pos, win.vel, win.force, win.k0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        binding.dpd_window_forward(sim.ctx, steps, ckpt, 2, nbins, prof, None)
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - ta)
        ta = time.perf_counter()
        g = binding.dpd_backward(sim.ctx, dldp, None)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - ta)
    sim.kernel_times(1)
    sim.step(20)
    kt = sim.kernel_times(0)
    sim.close()
    f_ms, b_ms = 1e3 * float(np.median(tf)), 1e3 * float(np.median(tb))
    log("adjoint window: %d particles, forward %.3f ms, backward %.3f ms (%d steps, ckpt %d), "
        "ratio %.2f" % (s.n, f_ms, b_ms, steps, ckpt, b_ms / f_ms))
    return {"workload": s.name, "particles": s.n, "fluid": s.n_fluid, "steps": steps,
            "ckpt": ckpt, "nbins": nbins, "forward_ms": f_ms, "backward_ms": b_ms,
            "ratio_backward_over_forward": b_ms / f_ms, "shape": list(shape),
            "grads": [float(x) for x in g],
            "step_kernel_ms": {k: v[0] / max(v[1], 1) for k, v in kt.items() if v[1]}}


def cpu_model():
    """Model name of the host CPU (first 'model name' of /proc/cpuinfo) and
    the number of logical CPUs."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s (%d logical CPUs)" % (name, os.cpu_count() or 0)


def reap_children():
    """End any child process this run started (none is expected: the legs
    use threads), so that nothing outlives the benchmark."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for k in kids:
        log("ending child process %d (%s)" % (k.pid, " ".join(k.cmdline()[:3])))
        k.terminate()
    psutil.wait_procs(kids, timeout=5)


def kernel_source_hash(files=("device.h", "kernels.hip", "api.hip")):
    """Hash of the sources that decide a stored traffic record: the step's
    kernels and the host code that launches them (tile tables and order)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1807_09896_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
    reap_children()
