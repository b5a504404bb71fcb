"""Throughput of the Newmark IMEX step on one MI355X.

Default workload: the 64^3-cell p=3 voided cube with 40 seeded spherical
voids (radii uniform in [0.02, 0.06], alpha_f = 1e-5, octree depth 2 on cut
cells, Ricker point source at 10 Hz in the centre of the bottom face, dt =
0.9 x the uncut-cell critical step), FP64 explicit state and FP64 implicit
block, 2000 steps (the workload's horizon).  A "step" is one Newmark IMEX
time step: explicit apply and CDM update of the d dofs, predictor, coupling
and cut-block right-hand side, the factorised solve of the c dofs by levels
of the nested-dissection factor, and the correction.

The timed region covers exactly --steps steps launched through the C ABI,
with the excitation table already resident in device memory, bracketed by
stream synchronisation.  Per-kernel durations come from HIP events that 32
further steps of the same run record on the library's stream right after
the timed region (imex_set_step_timing: events before and after each kernel
group of every step; HIP does not time event records captured in a graph,
so these steps are launched one by one), so every kernel runs after the
rest of a real step, as in the timed region.  The same kernels launched back
to back on their own (imex_time_kernel) are reported beside them as
kernels_us_isolated: there the working set stays partly in the 256 MB
Infinity Cache, which the rest of a step evicts.  The roofline uses the
isolated figures with an iterative or substepping solve, and when the
steps launched one by one fall behind the graph-launched ones (the three
groups' sum above 1.1 x the timed step: small steps, where launch gaps
would fall inside the events).  The roofline entry is the single-launch kernel with
the longest duration per step: the explicit kernel (stiffness apply and CDM
update) or the right-hand side (predictor and the K^cd, K^cc products); the
solve is a group of per-level launches and is reported beside them.  Its
HBM traffic comes from the committed FETCH_SIZE / WRITE_SIZE summary when
that was taken on the current kernel sources and the same workload, else it
is null.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROFILES = os.path.join(ROOT, "profiles")
TIMED_STEPS = 32  # steps after the timed region whose kernels are timed with events
METRIC = "DOF-updates/s per IMEX step at <=1e-6 rel L2 vs FP64 oracle; batched/learned vs plain"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(inf, fp_bytes, nnz_d, nnz_c):
    """Bytes each kernel must move per launch (documented in the design notes).

    explicit: FP64 two-step form: read u_n on active nodes, read u_{n-1} and write
              u_{n+1} over it on d nodes; FP32 increment form: read u_n, read and
              write the increment, write u_{n+1} (d nodes)
    rhs:      K^c values (8 B) and 4-byte column indices, u^c, v^c, a^c (24 B per c
              column), write rhs; the u^d_{n+1} gathers (one per K^cd nonzero, most of
              them cache hits on values the explicit step just wrote) are left out
    solve:    nested-dissection factor: every entry of L read by the forward and
              by the backward pass (16 B per entry of L), the update vectors
              written once and read once by the parent (16 B per update row) and
              the solution gathered at struct(s) in the backward pass (8 B per
              update row), the rhs read, y written and read (24 B per c row), the
              c state read and written (48 B) and u^c into the grid;
              dissected factor: the dense part and separator inverses once, the
              couplings Z_p once or twice (coupling_passes), envelope chains twice
              (forward and backward), rhs/solution and the c state, u^c into the
              grid; the sparse A_Sp of the wide form is left out
    """
    n_act, n_d, n_c = inf["n_active"], inf["n_d"], inf["n_c"]
    explicit = fp_bytes * (n_act + (2 if fp_bytes == 8 else 3) * n_d)
    rhs = 12 * (nnz_d + nnz_c) + 24 * n_c + 8 * n_c
    if inf.get("factor_form") == 1:
        solve = 16 * inf["nd_nnz_L"] + 24 * inf["nd_update_rows"] + 24 * n_c + 48 * n_c + fp_bytes * n_c
    else:
        solve = (8 * (inf["nnz_part_inv"] + inf["nnz_sep_inv"]) + 8 * inf["coupling_passes"] * inf["nnz_coupling"]
                 + 16 * inf["nnz_chain"] + 8 * 2 * n_c + 48 * n_c + fp_bytes * n_c)
    return {"explicit": explicit, "rhs": rhs, "solve": solve}


def cpu_info():
    """Model name of the host CPU and the core counts the process sees."""
    model = "unknown"
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
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(w, n_steps, replica=None):
    """The FP64 oracle (single thread) on the first n_steps of the workload.

    For the voided cubes the oracle cannot assemble the full problem (about
    1e9 nonzeros of K), so it runs the reduced replica given (same cell size,
    order, octree depth, void radii and voids per unit volume) and its rate
    per DOF-step is the extrapolated rate of the full cube."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import fcm, newmark
    from paper_2310_14712_amd import inputs
    run_w = replica or w
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        d = fcm.assemble(run_w)
        ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, d.dt)
        ft = inputs.ft_table(d.dt, n_steps, run_w.source_freq)
        st = ig.initial_state(np.zeros(d.n_grid), np.zeros(d.n_grid), ft[0])
        t0 = time.perf_counter()
        ig.run(st, ft, n_steps)
        el = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    n_act = len(d.active)
    us = el / (n_act * n_steps) * 1e6
    if replica is None:
        sample = (f"{w.name}: first {n_steps} of {w.steps} steps from rest, FP64 NumPy/SciPy, one thread; "
                  f"assembly and factorisation excluded; {el:.2f} s")
    else:
        sample = (f"extrapolated: {run_w.name} ({'x'.join(map(str, run_w.n_cells))} cells, {n_act} active dofs, "
                  f"{run_w.n_holes} voids; the cell size, order, octree depth, void radii and voids per volume of "
                  f"{w.name}), first {n_steps} steps from rest, FP64 NumPy/SciPy, one thread, assembly and "
                  f"factorisation excluded: {el:.2f} s = {us:.4f} us per DOF-step, applied to the full cube")
    return {"value": 1e6 / us, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle", "sample": sample,
            "us_per_dof_step": us, "extrapolated": replica is not None, **cpu_info()}


def large_grid_roofline(fp, stream, dim=2, p=4):
    """The explicit kernel alone on an uncut grid whose fields are far
    larger than the caches (2D: 2048 x 2048 cells at p = 4, 67M dofs; 3D:
    128^3 cells at p = 3, 57M dofs), autotuned, timed with HIP events on the
    library stream."""
    from paper_2310_14712_amd import imex, inputs
    n = 2048 if dim == 2 else 128
    w = inputs.Workload(name=f"uncut{n}_p{p}", dim=dim, n_cells=(n,) * dim, p=p,
                        source=(0.3, 0.4) if dim == 2 else (0.3, 0.4, 0.5))
    lib = imex.Imex(w, stream=stream.cuda_stream, explicit_fp=fp)
    lib.assemble()
    tiles = lib.autotune_tiles(5)
    inf = lib.info()
    lib.set_initial(None, None, 0.0)
    ms = lib.time_kernel(0, 50)
    fpb = fp // 8
    byt = fpb * (inf["n_active"] + (2 if fp == 64 else 3) * inf["n_d"])
    ach = byt / (ms * 1e-3) / 1e9
    lib.close()
    cells = "x".join([str(n)] * dim)
    return {"workload": f"uncut {cells} cells, p={p}, FP{fp} state", "kernel": "explicit", "bound": "hbm",
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "bytes_per_launch": byt, "launch_us": round(ms * 1e3, 2),
            "launch": {"tx": tiles[0], "ty": tiles[1], "lz": tiles[2], "mode": tiles[3]}}


def physical_points(w, n, seed):
    """n seeded points uniform in the box and outside every hole (points are
    drawn in the whole box and kept when physical, as in Section
    "Perforated plate")."""
    rng = np.random.default_rng(seed)
    ext = np.array(w.extent[:w.dim])
    pts = []
    while len(pts) < n:
        x = rng.uniform(0.0, 1.0, (n, w.dim)) * ext
        d = np.linalg.norm(x[:, None, :] - np.asarray(w.hole_centers)[None, :, :w.dim], axis=2)
        keep = np.all(d >= np.asarray(w.hole_radii)[None, :], axis=1)
        pts.extend(x[keep].tolist())
    return np.array(pts[:n])


def bench_accuracy(args):
    """Accuracy of the Newmark IMEX scheme and its comparators against a fine
    reference, with the relative L2 error of Section "Perforated plate":
    e_L2 = sqrt(sum_i (u(x_i) - u_ref(x_i))^2 / sum_i u_ref(x_i)^2) over
    8572 random points x_i in the physical domain, at the final time.

    Geometry: the 16 x 16-cell plate's (unit square, hole r = 0.2 at the
    centre, Ricker 10 Hz at (0.1, 0.5)), p = 4, on 16^2 and 32^2 cells, up to
    t = 1.  Schemes: Newmark IMEX at its own step (0.9 x the uncut-cell
    limit), central differences with the consistent and with the
    HRZ-lumped cut-cell mass (0.9 x their global critical steps), the fully
    implicit trapezoidal rule at the IMEX step, the substepping leap-frog
    (HRZ mass) at the IMEX step with the fewest substeps that keep the cut
    block stable, and IMEX at the central-difference step.  Reference: a
    separate finer run, 64^2 cells at p = 5 by central differences
    (consistent mass) at a quarter of its critical step.  The time is the
    GPU stepping wall time of each run (no sampling inside)."""
    import dataclasses
    import torch
    from paper_2310_14712_amd import imex, inputs
    T = 1.0
    base = inputs.config1()
    stream = torch.cuda.Stream()
    pts = physical_points(base, 8572, 2024)

    def run(n, scheme, p=4, safety=0.9, dt_force=None, m=0):
        w = dataclasses.replace(base, name=f"plate{n}_p{p}_1hole", n_cells=(n, n), p=p, explicit_fp=64)
        if scheme == "fully implicit":
            w = inputs.fully_implicit(w)
        if scheme in ("cdm hrz", "leap-frog"):
            w.cut_mass = "hrz"
        host = imex.Imex(w, device_mode=imex.HOST_ONLY)
        dt_max = host.info()["dt"] / w.cfl          # the uncut-cell critical step
        if scheme.startswith("cdm"):
            host.set_newmark_beta(0.0)
            host.assemble()
            dt_max = host.global_critical_step()
        if scheme == "leap-frog":
            host.set_newmark_beta(0.0)
            host.assemble()
            # substeps: the cut block's critical step (global step of the
            # central difference scheme with every d dof fixed is below it)
            dt_glob = host.global_critical_step()
            m = int(np.ceil(safety * dt_max / (safety * dt_glob)))
        host.close()
        dt = dt_force or safety * dt_max
        steps = int(np.ceil(T / dt))
        dt = T / steps
        lib = imex.Imex(w, stream=stream.cuda_stream, dt=dt)
        if scheme.startswith("cdm"):
            lib.set_newmark_beta(0.0)
        if scheme == "leap-frog":
            lib.set_leapfrog(m)
        lib.assemble()
        ft = inputs.ft_table(dt, steps, w.source_freq)
        ft_dev = torch.tensor(ft, dtype=torch.float64, device="cuda")
        lib.set_initial(None, None, ft[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.step(None, n_steps=steps, device_ptr=ft_dev.data_ptr())
        stream.synchronize()
        el = time.perf_counter() - t0
        vals = lib.sample(pts)
        lib.close()
        info = {"cells": n, "p": p, "scheme": scheme, "dt": dt, "steps": steps, "seconds": round(el, 4)}
        if m:
            info["substeps"] = m
        return vals, info

    ref, ref_info = run(64, "cdm", p=5, safety=0.25)
    results = []
    for n in (16, 32):
        runs = {}
        for scheme in ("imex", "cdm", "cdm hrz", "fully implicit", "leap-frog"):
            runs[scheme] = run(n, scheme)
        runs["imex at the cdm step"] = run(n, "imex", dt_force=runs["cdm"][1]["dt"])
        for name, (vals, info) in runs.items():
            info["scheme"] = name
            info["e_L2"] = float(np.sqrt(np.sum((vals - ref) ** 2) / np.sum(ref ** 2)))
            results.append(info)
            print(f"[bench] accuracy {info}", file=sys.stderr, flush=True)
    line = {"metric": "relative L2 error at t = 1 over random points of the physical domain vs a fine reference",
            "unit": "1", "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "plate with one hole (unit square, r = 0.2 at the centre, Ricker 10 Hz at "
                                   "(0.1, 0.5)), p = 4, t = 1, 8572 random physical points",
                       "reference": ref_info},
            "results": results}
    print(json.dumps(line))


def bench_batched(args):
    """64 independent 2D instances (33^2..128^2 cells, p = 2..6, 1..12 holes,
    FP32 explicit state), stepped together as a batch in its default form:
    one launch per kernel type per step over all instances (the explicit
    kernel once per order p), driven by per-instance argument tables, 32-step
    chunks captured in one graph.  Also times the same instances stepped one
    after another (each through its own autotuned 32-step graphs) as the
    plain reference, and the batch form that replays the instances' own
    graphs over 16 streams."""
    import torch
    from paper_2310_14712_amd import imex, inputs

    ws = inputs.config4_instances(64)
    stream = torch.cuda.Stream()
    t_setup = time.perf_counter()
    libs, tiles = [], []
    for w in ws:
        lib = imex.Imex(w, stream=stream.cuda_stream)
        lib.assemble()
        tiles.append(lib.autotune_tiles(20))
        libs.append(lib)
    t_setup = time.perf_counter() - t_setup
    total = args.warmup + args.steps
    infs = [lib.info() for lib in libs]
    fts = [torch.tensor(inputs.ft_table(inf["dt"], total, w.source_freq), dtype=torch.float64, device="cuda")
           for inf, w in zip(infs, ws)]
    n_act = sum(inf["n_active"] for inf in infs)

    def reset():
        for lib, ft in zip(libs, fts):
            lib.set_initial(None, None, float(ft[0]))
        torch.cuda.synchronize()

    # plain: one instance after another
    reset()
    for lib, ft in zip(libs, fts):
        lib.step(None, n_steps=args.warmup, device_ptr=ft.data_ptr())
    stream.synchronize()
    t0 = time.perf_counter()
    for lib, ft in zip(libs, fts):
        lib.step(None, n_steps=args.steps, device_ptr=ft.data_ptr() + 8 * args.warmup)
    stream.synchronize()
    el_plain = time.perf_counter() - t0
    def run_batch(lanes_env):
        reset()
        if lanes_env is not None:
            os.environ["IMEX_BATCH_LANES"] = lanes_env
        try:
            batch = imex.Batch(libs, stream=stream.cuda_stream)
        finally:
            os.environ.pop("IMEX_BATCH_LANES", None)
        batch.step(args.warmup, device_ptrs=[ft.data_ptr() for ft in fts])
        stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(args.steps, device_ptrs=[ft.data_ptr() + 8 * args.warmup for ft in fts])
        stream.synchronize()
        el_ = time.perf_counter() - t0
        form_ = batch.form()
        batch.close()
        return el_, form_

    el_lanes, _ = run_batch("16")
    el, form = run_batch(None)
    print(f"[bench] batch: {args.steps} steps in {el:.4f} s (form {form}; lanes form {el_lanes:.4f} s; "
          f"one by one: {el_plain:.4f} s)", file=sys.stderr, flush=True)
    # explicit kernels of all instances: algorithmic bytes over summed durations
    byt, ms = 0.0, 0.0
    for lib, inf in zip(libs, infs):
        lib.set_initial(None, None, 0.0)
        ms += lib.time_kernel(0, max(10, args.kernel_reps // 10))
        byt += 4 * (inf["n_active"] + 3 * inf["n_d"])
    ach = byt / (ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": n_act * args.steps / el,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config4: 64 independent 2D instances, 33^2..128^2 cells, p=2..6, 1..12 seeded "
                               "holes, FP32 explicit state, FP64 implicit block, batched kernels (one launch per "
                               "kernel type and step over all instances), 32-step graphs",
                   "batch_form": ["one graph, a branch per instance", "instances' graphs over 16 streams",
                                  "batched kernels"][form],
                   "lanes_value": n_act * args.steps / el_lanes,
                   "n_active": n_act, "n_c": sum(inf["n_c"] for inf in infs), "instances": len(ws),
                   "setup_s": round(t_setup, 3),
                   "plain_value": n_act * args.steps / el_plain,
                   "batched_over_plain": el_plain / el,
                   "tiles": [list(t[:2]) for t in tiles]},
        "roofline": {"bound": "hbm", "kernel": "explicit (all instances, one by one)", "achieved": round(ach, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                     "traffic": None, "bytes_per_launch": byt, "launch_us": round(ms * 1e3, 3)},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="config3", choices=["config1", "config2", "config3", "config4", "config5"],
                    help="config4 runs the 64-instance batch (see bench_batched)")
    ap.add_argument("--fp", type=int, default=64,
                    help="explicit-part state precision (64; 32 stores the grid state in FP32)")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps of the CPU baseline (default 2000 on the plates, 300 on the cube replicas)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solver", default="cholesky", choices=["cholesky", "jacobi", "block", "mlp"],
                    help="implicit-block solver of the timed steps (iterative ones: flexible CG to 1e-10)")
    ap.add_argument("--train-epochs", type=int, default=60,
                    help="--solver mlp: epochs over the vectors collected during the warm-up steps")
    ap.add_argument("--train-batch", type=int, default=8, help="--solver mlp: vectors per training batch")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the explicit-kernel measurement on a 2048x2048-cell uncut grid")
    ap.add_argument("--accuracy", action="store_true",
                    help="receiver accuracy of IMEX and the comparators against a fine reference (config1 geometry)")
    ap.add_argument("--cdm", action="store_true",
                    help="comparator: central differences on all dofs at the global critical step")
    ap.add_argument("--hrz", action="store_true",
                    help="with --cdm: HRZ-lumped cut-cell masses (the lumped-mass CDM comparator)")
    ap.add_argument("--leapfrog", action="store_true",
                    help="comparator: leap-frog with m substeps on the cut-cell dofs (HRZ cut mass), m the "
                         "smallest with dt / m below cfl x the global critical step")
    ap.add_argument("--fully-implicit", action="store_true",
                    help="comparator: every cell in the implicit block (trapezoidal Newmark on all dofs)")
    ap.add_argument("--launch", default=None, metavar="TX,TY,LZ,MODE",
                    help="fixed explicit launch shape instead of the autotuner's choice")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="finish with one device-to-device copy of MIB MiB (counter calibration runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; runs on more than one GPU are not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_14712_amd import imex, inputs

    if args.accuracy:
        return bench_accuracy(args)
    if args.config == "config4":
        return bench_batched(args)
    w = getattr(inputs, args.config)()
    if args.fully_implicit:
        w = inputs.fully_implicit(w)
    if args.hrz or args.leapfrog:
        w.cut_mass = "hrz"
    w.explicit_fp = args.fp
    stream = torch.cuda.Stream()
    t_setup = time.perf_counter()
    if args.launch:
        # a fixed launch shape of the explicit kernel (counter runs use the
        # shape an earlier autotuned run chose)
        tiles = [int(v) for v in args.launch.split(",")]
        for k, v in zip(("IMEX_TX", "IMEX_TY", "IMEX_LZ", "IMEX_EXPLICIT_MODE"), tiles):
            os.environ[k] = str(v)
    dt_imex = dt_global = None
    lts_m = None
    if args.leapfrog:
        host = imex.Imex(w, device_mode=imex.HOST_ONLY)
        dt_imex = host.info()["dt"]
        host.assemble()
        dt_global = host.global_critical_step()
        host.close()
        lts_m = int(np.ceil(dt_imex / (w.cfl * dt_global)))
        lib = imex.Imex(w, stream=stream.cuda_stream)
        lib.set_leapfrog(lts_m)
    elif args.cdm:
        # the comparator runs at the global critical step (cfl of the workload)
        host = imex.Imex(w, device_mode=imex.HOST_ONLY)
        dt_imex = host.info()["dt"]
        host.assemble()
        dt_global = host.global_critical_step()
        host.close()
        lib = imex.Imex(w, stream=stream.cuda_stream, dt=w.cfl * dt_global)
        lib.set_newmark_beta(0.0)
    else:
        lib = imex.Imex(w, stream=stream.cuda_stream)
    lib.assemble()
    if not args.launch:
        tiles = lib.autotune_tiles(50)   # launch shape of the explicit kernel (does not change results)
    t_setup = time.perf_counter() - t_setup
    inf = lib.info()
    dt = inf["dt"]
    total = args.warmup + args.steps + TIMED_STEPS
    ft = inputs.ft_table(dt, total, w.source_freq)
    ft_dev = torch.tensor(ft, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lib.set_initial(None, None, ft[0])
    solver = {"cholesky": imex.SOLVER_CHOLESKY, "jacobi": imex.SOLVER_PCG_JACOBI, "block": imex.SOLVER_PCG_BLOCK,
              "mlp": imex.SOLVER_PCG_MLP}[args.solver]
    train = None
    if args.solver == "mlp":
        # the warm-up steps (factorised solve) supply the training vectors
        sh = lib.mlp_shape()
        lib.mlp_set_weights(inputs.mlp_init(sh["inputs"], sh["hidden"], sh["outputs"], 11, 0.01))
        lib.mlp_collect(2 * args.warmup)
    # warm-up (also captures the step graphs)
    lib.step(None, n_steps=args.warmup, device_ptr=ft_dev.data_ptr())
    stream.synchronize()
    print(f"[bench] {args.warmup} warm-up steps done", file=sys.stderr, flush=True)
    if args.solver == "mlp":
        lib.mlp_collect(0)
        print(f"[bench] training on {lib.mlp_shape()['collected']} vectors", file=sys.stderr, flush=True)
        t_tr = time.perf_counter()
        ep = 0
        while ep < args.train_epochs:   # in chunks of 5 epochs (Adam's state carries over), with progress lines
            k = min(5, args.train_epochs - ep)
            loss = lib.mlp_train(k, args.train_batch, 1e-3, 1 + ep)
            ep += k
            print(f"[bench] epoch {ep}: loss {loss:.4g}, {time.perf_counter() - t_tr:.1f} s", file=sys.stderr,
                  flush=True)
        train = {"vectors": lib.mlp_shape()["collected"], "epochs": args.train_epochs,
                 "vectors_per_batch": args.train_batch, "loss": loss,
                 "seconds": round(time.perf_counter() - t_tr, 3)}
    if solver != imex.SOLVER_CHOLESKY:
        lib.set_solver(solver, 1e-10, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if solver == imex.SOLVER_CHOLESKY:
        lib.step(None, n_steps=args.steps, device_ptr=ft_dev.data_ptr() + 8 * args.warmup)
    else:
        # iterative solves synchronise with the host anyway: steps in chunks
        # with a progress line each
        done = 0
        while done < args.steps:
            k = min(250, args.steps - done)
            lib.step(None, n_steps=k, device_ptr=ft_dev.data_ptr() + 8 * (args.warmup + done))
            done += k
            print(f"[bench] {done} / {args.steps} steps, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    stream.synchronize()
    el = time.perf_counter() - t0
    print(f"[bench] {w.name}: {args.steps} steps in {el:.4f} s", file=sys.stderr, flush=True)
    in_step = in_step_raw = None
    if solver == imex.SOLVER_CHOLESKY and not args.leapfrog:
        # per-kernel events in TIMED_STEPS further steps (factorised solve)
        lib.set_step_timing(True)
        lib.step(None, n_steps=TIMED_STEPS, device_ptr=ft_dev.data_ptr() + 8 * (args.warmup + args.steps))
        in_step = in_step_raw = lib.step_timing()
        lib.set_step_timing(False)
        # steps launched one by one must keep the GPU as busy as the graphs:
        # else launch gaps fall inside the events (small steps), and the
        # back-to-back figures stand in
        if sum(in_step.values()) > 1.1 * el / args.steps * 1e3:
            in_step = None
    solver_stats = lib.solver_stats() if solver != imex.SOLVER_CHOLESKY else None
    accuracy = None
    if solver != imex.SOLVER_CHOLESKY:
        # the same steps with the factorised solve: the iterative run's field
        # against it (the 1e-6 accuracy bar of the metric), and its time
        ref = imex.Imex(w, stream=stream.cuda_stream)
        ref.assemble()
        ref.set_initial(None, None, ft[0])
        ref.step(None, n_steps=args.warmup, device_ptr=ft_dev.data_ptr())
        stream.synchronize()
        t0 = time.perf_counter()
        ref.step(None, n_steps=args.steps, device_ptr=ft_dev.data_ptr() + 8 * args.warmup)
        stream.synchronize()
        el_ref = time.perf_counter() - t0
        u_it, u_ref = lib.read(imex.FIELD_U), ref.read(imex.FIELD_U)
        accuracy = {"rel_l2_u_vs_factor": float(np.linalg.norm(u_it - u_ref) / np.linalg.norm(u_ref)),
                    "factor_ms_per_step": el_ref * 1e3 / args.steps,
                    "iterative_ms_per_step": el * 1e3 / args.steps}
        ref.close()

    # per-kernel durations (HIP events on the library stream)
    rp, cols, _ = lib.export_csr(imex.CSR_KC)
    cn = lib.export_index(imex.INDEX_C_NODES)
    is_c = np.zeros(inf["n_grid"], dtype=bool)
    is_c[cn] = True
    nnz_c = int(is_c[cols].sum())
    nnz_d = len(cols) - nnz_c
    fpb = 8 if args.fp == 64 else 4
    algo = algorithmic_bytes(inf, fpb, nnz_d, nnz_c)
    kernels = {}
    for name, k in (("explicit", 0), ("rhs", 1), ("solve", 2)):
        if k > 0 and inf["n_c"] == 0:
            continue
        lib.set_initial(None, None, ft[0])
        ms_iso = lib.time_kernel(k, args.kernel_reps)
        ms = in_step[name] if in_step else ms_iso
        kernels[name] = {"ms": ms, "ms_isolated": ms_iso, "bytes": algo[name],
                         "GBps": algo[name] / (ms * 1e-3) / 1e9}
    # the single-launch kernel with the longest duration per step (the
    # explicit kernel or the right-hand side; the solve is a group of
    # per-level launches, reported beside them)
    single = [k for k in ("explicit", "rhs") if k in kernels and algo[k] > 0 and (k != "explicit" or inf["n_d"] > 0)]
    dom = max(single, key=lambda k: kernels[k]["ms"]) if single else "solve"
    ach = kernels[dom]["GBps"]
    workload = (f"{w.name}: {w.dim}D {'x'.join(map(str, w.n_cells))} cells, p={w.p}, "
                f"{w.n_holes} seeded holes, alpha_f={w.alpha_f}, tree depth {w.tree_depth}, "
                f"Ricker {w.source_freq} Hz point source, cfl {w.cfl}, FP{args.fp} explicit state"
                + (", central difference comparator" if args.cdm else "")
                + (", HRZ-lumped cut-cell mass" if args.hrz else ""))
    traffic = None
    # HBM traffic from a committed counter summary of this workload, taken
    # with the current kernel sources
    from paper_2310_14712_amd import profiling
    for fn in sorted(os.listdir(PROFILES)):
        if not fn.endswith("_traffic.json"):
            continue
        try:
            with open(os.path.join(PROFILES, fn)) as f:
                tr = json.load(f)
            if (tr["kernels_sha256"] == profiling.kernel_source_sha256() and tr["workload"] == workload
                    and tr.get("kernel_key", "explicit") == dom):
                traffic = tr["traffic_bytes_per_launch"]
        except (OSError, KeyError, ValueError):
            continue
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": traffic,
            "bytes_per_launch": algo[dom], "launch_us": round(kernels[dom]["ms"] * 1e3, 3),
            "timing": (f"HIP events around the kernels of {TIMED_STEPS} steps right after the timed region"
                       if in_step else
                       "HIP events around back-to-back launches of each kernel alone"),
            "kernels_us": {k: round(v["ms"] * 1e3, 3) for k, v in kernels.items()},
            "kernels_us_isolated": {k: round(v["ms_isolated"] * 1e3, 3) for k, v in kernels.items()},
            **({"kernels_us_steps_one_by_one": {k: round(v * 1e3, 3) for k, v in in_step_raw.items()}}
               if in_step_raw and not in_step else {}),
            "kernels_bytes": {k: v["bytes"] for k, v in kernels.items()},
            "kernels_GBps": {k: round(v["GBps"], 2) for k, v in kernels.items()}}
    line = {
        "metric": METRIC,
        "value": inf["n_active"] * args.steps / el,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n_active": inf["n_active"], "n_d": inf["n_d"], "n_c": inf["n_c"],
                   "n_components": inf["n_components"], "nnz_factor": inf["nnz_factor"],
                   "factor_values": ({k: inf[k] for k in ("nd_supernodes", "nd_levels", "nd_nnz_L",
                                                          "nd_update_rows", "nd_max_m", "nd_max_mk")}
                                     if inf.get("factor_form") == 1 else
                                     {k: inf[k] for k in ("nnz_part_inv", "nnz_coupling", "nnz_sep_inv", "nnz_chain",
                                                          "coupling_passes")}),
                   "dt": dt, "setup_s": round(t_setup, 3), "solver": args.solver,
                   **({"scheme": "leap-frog, m substeps of dt / m on the cut-cell dofs (HRZ cut mass)",
                       "substeps": lts_m, "dt_global_crit": dt_global} if args.leapfrog else {}),
                   **({"scheme": "central differences on all dofs (beta = 0 on the c block), "
                                 "dt = cfl x global critical step",
                       "dt_global_crit": dt_global, "dt_imex": dt_imex,
                       "steps_per_imex_step": dt_imex / dt} if args.cdm else {}),
                   "explicit_launch": {"tx": tiles[0], "ty": tiles[1], "lz": tiles[2],
                                       "mode": ["lds tiles", "strips", "strips, staged loads",
                                                "lds tiles, 128 threads", "lds tiles, 512 threads",
                                                "tensor-product form"][tiles[3]],
                                       "arg": ",".join(map(str, tiles)), "autotuned": not args.launch}},
        "roofline": roof,
    }
    if not args.no_large:
        line["roofline_large"] = large_grid_roofline(args.fp, stream, w.dim, 4 if w.dim == 2 else 3)
    if solver_stats is not None:
        line["config"]["solver_stats"] = {k: solver_stats[k] for k in ("solves", "iterations", "fallbacks")}
        line["config"]["solver_stats"]["mean_iterations"] = solver_stats["iterations"] / max(1, solver_stats["solves"])
        line["config"]["against_factor"] = accuracy
        if train:
            line["config"]["training"] = train
    if not args.no_cpu_baseline:
        replica = None
        if args.config in ("config3", "config5"):
            replica = getattr(inputs, args.config + "_replica")()
        cpu_steps = args.cpu_steps or (300 if replica is not None else 2000)
        line["cpu_baseline"] = cpu_baseline(w, cpu_steps, replica)
    print(json.dumps(line), flush=True)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.copy_calibration} MiB done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
