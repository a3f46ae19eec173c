#!/usr/bin/env python3
"""Benchmark of the SLLBM hot path on one MI355X.

One "step" is the whole per-time-step update of the state over the grid: the
collision kernel (moments, transport coefficients, equilibria,
quasi-equilibrium term, relaxation of all 90 populations of every node) and
the streaming kernel (the order-p semi-Lagrangian interpolation of all 90
populations).  The headline workload is the largest single-GPU grid of the
configurations: the FP64 compressible Taylor-Green vortex on 64^3 cells of
order 4 (256^3 nodes), Ma 1.25, Re 1600, CFL 10 with the seeded velocity
modes.  The FP32-mixed step on the same grid and the FP64 step on 16^3 cells
(64^3 nodes) are reported beside it.  Every timing is the median of --reps
repetitions of K steps, each from the same post-warmup state.
``--workload riemann`` (or ``sod``) measures the two-dimensional D2Q19 step
instead: 38 populations per node, case 12 of the 2-D Riemann problems on
128^2 cells of order 4 (512^2 nodes).

Prints ONE JSON line (see the ``--help`` of the options).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
Q = 45

# sources that determine each timed kernel, besides the headers of csrc/ that
# they include (a change in any of them voids committed counters)
KERNEL_SOURCES = {
    "k_stream_z": ("stream.hip", "tables.cpp"),
    "k_stream_graded": ("stream_graded.hip", "tables.cpp"),
    "k_collide": ("kernels.hip", "collision.h", "velset.h"),
    "k_stream_y": ("stream2d.hip", "tables.cpp"),
    "k_stream_mapped": ("stream_mapped.hip", "tables_mapped.cpp"),
}


def _code_only(text):
    """Source text without comments and with whitespace collapsed (a comment
    edit does not change the kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_files(kernel):
    """The kernel's sources and, transitively, the csrc/ headers they include."""
    csrc = os.path.join(ROOT, "paper_2012_05537_amd", "csrc")
    seen, todo = [], list(KERNEL_SOURCES[kernel])
    while todo:
        f = todo.pop(0)
        path = os.path.join(csrc, f)
        if f in seen or not os.path.exists(path):     # the public header lives in include/
            continue
        seen.append(f)
        with open(path, encoding="utf-8") as fh:
            todo += re.findall(r'^\s*#include "([^"]+)"', fh.read(), flags=re.M)
    return sorted(seen)


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for f in kernel_source_files(kernel):
        with open(os.path.join(ROOT, "paper_2012_05537_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(f"{kernel}:{workload}:{dtype}")
    if not rec or rec.get("kernel_source") != kernel_source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def run_gpu(args, wl, precision, mesh="equal"):
    import torch
    from paper_2012_05537_amd import inputs
    from paper_2012_05537_amd.sllbm import SLLBM

    ctx = SLLBM(wl["n_el"], wl["p"], wl["dt"], wl["mu_inf"], gamma=wl["gamma"], prandtl=wl["Pr"],
                precision=precision)
    if mesh == "graded":
        w = inputs.graded_widths(wl["n_el"], amplitude=inputs.GRADED["amplitude"])
        ctx.set_mesh(w, w, w)
    xs, ys, zs = (t.numpy() for t in ctx.node_coords())
    md = wl.get("modes")
    modes = inputs.fourier_modes(md["seed"], md["count"], wl["Ma"], wl["gamma"], md["scale"]) if md else None
    rho, u, T = inputs.perturbed_tgv(xs, ys, zs, wl["Ma"], wl["gamma"], modes)
    dev = ctx.device
    ctx.init_equilibrium(torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev))
    del rho, u, T
    table_bytes = 0
    if mesh == "distorted":
        X, Y, Z = inputs.mesh(xs, ys, zs)
        ctx.set_displacement(inputs.distortion(X, Y, Z, 2 * math.pi / wl["n_el"], inputs.DISTORTED["amplitude"]))
        elem = 8 if precision == 0 else 4
        table_bytes = Q * ctx.nodes * (4 + 3 * elem)   # departure cell and local coordinates per velocity and node
    kern = {"graded": "k_stream_graded", "distorted": "k_stream_mapped"}.get(mesh, "k_stream_z")
    return measure_steps(args, ctx, kern, table_bytes)


def run_gpu_2d(args, wl, precision):
    """The two-dimensional (D2Q19) step on the periodic Sod tube or Riemann case 12."""
    import torch
    from paper_2012_05537_amd import inputs
    from paper_2012_05537_amd.sllbm import SLLBM, D2Q19, CONSTANT

    ctx = SLLBM(wl["n_el"], wl["p"], wl["dt"], wl["mu_inf"], gamma=wl["gamma"], prandtl=wl["Pr"],
                length=wl["length"], viscosity_law=CONSTANT, precision=precision, velocity_set=D2Q19)
    xs, ys = (t.numpy() for t in ctx.node_coords())
    rho, u, T = (inputs.sod_fields if wl["name"] == "sod" else inputs.riemann_fields)(xs, ys)
    dev = ctx.device
    ctx.init_equilibrium(torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev))
    return measure_steps(args, ctx, "k_stream_y")


def measure_steps(args, ctx, stream_kernel, table_bytes=0):
    """Wall clock of args.steps steps, then kernel durations from HIP events."""
    import torch
    dev = ctx.device
    precision = 0 if ctx.dtype == torch.float64 else 1
    if args.copy_calibration:
        # a plain copy kernel of one state's size (reads B, writes B; an elementwise
        # kernel, not a DMA copy), so that a counter run sees the HBM counters of a
        # kernel with known traffic beside the step's kernels
        src = torch.ones(ctx.state_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        ctx.step(1)
    start = ctx.get_state()
    walls = []
    for _ in range(max(1, args.reps)):
        # every repetition times the same K steps from the post-warmup state
        ctx.set_state(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.step(1)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    wall = sorted(walls)[len(walls) // 2]
    try:
        tot = ctx.totals()
        ok = all(math.isfinite(v) for v in tot)
    except RuntimeError:                 # non-finite totals: the flow itself blew up
        tot, ok = None, False
    # the same K steps again from the same state with HIP events around every
    # kernel launch, on the library's stream (kept out of the wall-clock region:
    # each event record adds a few microseconds between the launches)
    ctx.set_state(start)
    ctx.set_kernel_timing(True)
    for _ in range(args.steps):
        ctx.step(1)
    kt = ctx.kernel_times()
    ctx.set_kernel_timing(False)
    del start
    nodes = ctx.nodes
    elem = 8 if precision == 0 else 4
    bytes_per_launch = 2 * 2 * ctx.q * nodes * elem      # each kernel reads 2Q and writes 2Q values per node
    ctx.close()
    kernels = {name: {"ms": ms / max(n, 1), "launches": n, "bytes": b} for name, (ms, n), b in
               (("k_collide", kt["collide"], bytes_per_launch),
                (stream_kernel, kt["stream"], bytes_per_launch + table_bytes))}
    return dict(nodes=nodes, wall=wall, walls=walls, kernels=kernels, bytes=bytes_per_launch, finite=ok, totals=tot)


def run_adjoint(wl, precision, mesh="equal"):
    """Wall time of a checkpointed rollout gradient of the workload (forward
    rollout with checkpoints, then the reverse sweep with segment replay), and
    the ratio backward / forward."""
    import numpy as np
    import torch
    from paper_2012_05537_amd import inputs
    from paper_2012_05537_amd.adjoint import Rollout
    from paper_2012_05537_amd.sllbm import SLLBM

    ctx = SLLBM(wl["n_el"], wl["p"], wl["dt"], wl["mu_inf"], gamma=wl["gamma"], prandtl=wl["Pr"],
                precision=precision)
    if mesh == "graded":
        w = inputs.graded_widths(wl["n_el"], amplitude=inputs.GRADED["amplitude"])
        ctx.set_mesh(w, w, w)
    xs, ys, zs = (t.numpy() for t in ctx.node_coords())
    if mesh == "distorted":
        X, Y, Z = inputs.mesh(xs, ys, zs)
        ctx.set_displacement(inputs.distortion(X, Y, Z, 2 * math.pi / wl["n_el"], inputs.DISTORTED["amplitude"]))
    md = wl.get("modes") or dict(seed=2012, count=16, scale=0.01)
    modes = inputs.fourier_modes(md["seed"], md["count"], wl["Ma"], wl["gamma"], md["scale"])
    rho, u, T = inputs.tgv_fields(xs, ys, zs, wl["Ma"], wl["gamma"])
    B = inputs.mode_basis(xs, ys, zs, modes)
    steps = wl["steps"]
    roll = Rollout(ctx, rho, u, T, B, steps, checkpoint=wl.get("checkpoint", 10))
    del B
    amps = torch.tensor(np.array([m[3] for m in modes]), dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(wl["mu_inf"], dtype=torch.float64, requires_grad=True)
    roll(amps, mu).backward()                     # warm-up (allocations, first launches)
    amps.grad = None
    mu.grad = None
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    L = roll(amps, mu)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # checkpoints, segment record and adjoint buffers (torch) plus the library's two state buffers
    peak_gb = (torch.cuda.max_memory_allocated() + 2 * ctx.state_bytes) / 1e9
    ctx.close()
    cells = {"equal": "cells", "graded": "cosine-graded cells",
             "distorted": f"distorted cells (displacement {inputs.DISTORTED['amplitude']} h)"}[mesh]
    return {"workload": f"{wl['name']}{'' if mesh == 'equal' else '-' + mesh}: {wl['n_el']}^3 {cells} p={wl['p']} "
                        f"({ctx.nodes} nodes), {steps} steps, "
                        f"{len(modes)} modes + mu_inf, checkpoint {wl.get('checkpoint', 10)}",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "loss": L.item(), "grad_finite": bool(torch.isfinite(amps.grad).all() and math.isfinite(mu.grad.item())),
            "device_memory_GB": peak_gb}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _time_oracle(O, step, nodes, budget_s, what):
    """Whole-grid oracle steps (step() advances the state by one) until about
    budget_s seconds have run on all the oracle's OpenMP threads, then on one
    thread for about half that (at least one step)."""
    lib = O._lib()
    threads = int(lib.omp_get_max_threads())
    out = {}
    for n_threads, budget in ((threads, budget_s), (1, 0.5 * budget_s)):
        lib.omp_set_num_threads(n_threads)
        steps = 0
        t0 = time.perf_counter()
        while True:
            step()
            steps += 1
            el = time.perf_counter() - t0
            if el > budget or el / steps * (steps + 1) > 2.0 * budget:
                break
        out[n_threads] = (nodes * steps / el, steps, el)
    lib.omp_set_num_threads(threads)
    value, steps, el = out[threads]
    return dict(value=value, unit="node-updates/s", cores=threads, kind="oracle",
                sample=f"{steps} whole-grid FP64 {what} step(s) of the same workload ({nodes} nodes), {el:.1f} s",
                value_one_core=out[1][0], sample_one_core=f"{out[1][1]} step(s), {out[1][2]:.1f} s",
                cpu_model=_cpu_model())


def cpu_baseline(wl, budget_s, graded=False):
    """The FP64 oracle on the host cores: whole-grid steps of the same workload
    (same grid, same mesh, same parameters) until about budget_s seconds have
    run; then the same on one core."""
    from oracle import oracle as O
    from paper_2012_05537_amd import inputs

    widths = None
    if graded:
        w = inputs.graded_widths(wl["n_el"], amplitude=inputs.GRADED["amplitude"])
        widths = [w, w, w]
    cfg = O.make_cfg(wl["n_el"], wl["p"], wl["dt"], wl["mu_inf"], gamma=wl["gamma"], prandtl=wl["Pr"],
                     widths=widths)
    rho, u, T = inputs.tgv_fields(*O.node_coords(cfg), wl["Ma"], wl["gamma"])
    st = list(O.init_equilibrium(cfg, rho, u, T))

    def step():
        st[0], st[1] = O.step(cfg, st[0], st[1], 1)
    return _time_oracle(O, step, O.num_nodes(cfg), budget_s, "oracle")


def cpu_baseline_2d(wl, budget_s):
    """The 2-D FP64 oracle on the host cores: whole-grid steps of the same
    workload, then the same on one core."""
    from oracle import oracle2d as O
    from paper_2012_05537_amd import inputs

    cfg = O.make_cfg(wl["n_el"], wl["p"], wl["dt"], wl["mu_inf"], gamma=wl["gamma"], prandtl=wl["Pr"],
                     length=wl["length"], viscosity_law=O.CONSTANT)
    x, y = O.node_coords(cfg)
    rho, u, T = (inputs.sod_fields if wl["name"] == "sod" else inputs.riemann_fields)(x, y)
    st = list(O.init_equilibrium(cfg, rho, u, T))

    def step():
        st[0], st[1] = O.step(cfg, st[0], st[1], 1)
    return _time_oracle(O, step, O.num_nodes(cfg), budget_s, "2-D oracle")


def workload_2d(name):
    from paper_2012_05537_amd import inputs
    w = dict(inputs.WORKLOADS_2D[name])
    w["name"] = name
    return w


def copy_bandwidth(state_bytes, reps=5):
    """GB/s of a plain elementwise copy kernel (torch mul by 1.0) of one
    state's size, read + write, median over reps launches timed with events
    on torch's stream (where the copy runs)."""
    import statistics
    import torch
    n = max(1, state_bytes // 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(src, 1.0, out=dst)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (statistics.median(times) * 1e-3) / 1e9


def measure_line(args, wl, wkey, prec_name, two_d, mesh):
    """Timings of one workload and precision: (summary dict, raw record)."""
    from paper_2012_05537_amd import inputs
    precision = 0 if prec_name == "fp64" else 1
    r = run_gpu_2d(args, wl, precision) if two_d else run_gpu(args, wl, precision, mesh)
    dom = max(r["kernels"], key=lambda k: r["kernels"][k]["ms"])
    kms = r["kernels"][dom]["ms"]
    dom_bytes = r["kernels"][dom]["bytes"]
    achieved = dom_bytes / (kms * 1e-3) / 1e9
    kernels = {}
    for k, v in r["kernels"].items():
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None
        kernels[k] = {"ms_per_launch": v["ms"], "launches": v["launches"], "algorithmic_GBps": gbs,
                      "traffic": measured_traffic(k, wkey, prec_name)}
    if two_d:
        nx, ny = wl["n_el"]
        workload = (f"{wkey}: {'periodic double Sod tube' if wkey == 'sod' else 'Riemann case 12'} "
                    f"{nx}x{ny} cells p={wl['p']} ({r['nodes']} nodes), D2Q19, dt {wl['dt']}, "
                    f"mu {wl['mu_inf']}, {prec_name}")
    else:
        mdesc = {"equal": "cells", "graded": "cosine-graded cells (a = 0.3)",
                 "distorted": f"distorted cells (displacement {inputs.DISTORTED['amplitude']} h)"}[mesh]
        modes = " + 16 seeded velocity modes" if wl.get("modes") else ""
        workload = (f"{wkey}: TGV{modes} {wl['n_el']}^3 {mdesc} p={wl['p']} "
                    f"({r['nodes']} nodes), Ma {wl['Ma']}, Re {wl['Re']}, CFL {wl['cfl']}, {prec_name}")
    step_s = r["wall"] / args.steps
    copy_gbs = copy_bandwidth(r["bytes"] // 2)
    line = {
        "workload": workload,
        "value": r["nodes"] / step_s,
        "ms_per_step": step_s * 1e3,
        "ms_per_step_reps": [w * 1e3 / args.steps for w in r["walls"]],
        "dtype": "f64" if precision == 0 else "f32 (f64 moments)",
        "nodes": r["nodes"], "order": wl["p"], "cfl": wl.get("cfl"), "dt": wl["dt"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": kernels[dom]["traffic"],
                     "kernel": dom, "kernel_ms": kms, "algorithmic_bytes_per_launch": dom_bytes,
                     "step_frac": r["bytes"] / step_s / 1e9 / HBM_PEAK_GBS,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "kernels": kernels,
        "finite": r["finite"],
    }
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=5, help="repetitions of the K timed steps (median reported)")
    ap.add_argument("--workload", default=None,
                    help="workload key (c1..c5; sod or riemann: 2-D D2Q19); default c5 on equal cells, "
                         "c2 on graded or distorted cells")
    ap.add_argument("--cfl", type=float, default=None, help="CFL override (default: the workload's own)")
    ap.add_argument("--mesh", choices=["equal", "graded", "distorted"], default="equal",
                    help="equal cells, the cosine-graded cells of every axis (streaming on per-node tables), or "
                         "the smoothly distorted cells of sllbm_set_displacement (no cpu_baseline)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary lines (FP32-mixed on the same grid; with the default workload also "
                         "FP64 on 64^3 and 128^3 nodes, on the graded and distorted 64^3-node meshes and on the 2-D "
                         "Riemann workload)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-workload", default="c4",
                    help="workload whose rollout gradient is timed for the adjoint/forward ratio ('none' to skip)")
    ap.add_argument("--adjoint-cfl", type=float, default=None, help="CFL override of the adjoint workload")
    ap.add_argument("--adjoint-steps", type=int, default=None, help="rollout length override of the adjoint workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run three plain copies of one state's size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the step would shard "
              "as a periodic block decomposition with one halo exchange per step); run with --gpus 1",
              file=sys.stderr)
        return 2

    from paper_2012_05537_amd import inputs
    if args.workload is None:
        args.workload = "c5" if args.mesh == "equal" else "c2"
    two_d = args.workload in inputs.WORKLOADS_2D
    if two_d and args.mesh != "equal":
        print("the two-dimensional workloads use equal cells", file=sys.stderr)
        return 2
    over = {} if args.cfl is None else {"cfl": args.cfl}
    wl = workload_2d(args.workload) if two_d else inputs.workload(args.workload, **over)
    wkey = args.workload if args.mesh == "equal" else f"{args.workload}-{args.mesh}"
    head = measure_line(args, wl, wkey, args.precision, two_d, args.mesh)
    if two_d:
        data = "synthetic: piecewise-constant Riemann initial states (periodic stand-in)"
    else:
        data = "synthetic: closed-form compressible Taylor-Green vortex"
    out = {
        "metric": "node-updates/s (D2V19 f+g)" if two_d else "node-updates/s (D3V45 f+g)",
        "value": head["value"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": data,
        "config": {"workload": head["workload"], "nodes": head["nodes"], "order": head["order"],
                   "cfl": head["cfl"], "dt": head["dt"], "parallelism": "single GPU",
                   "timing": f"median of {args.reps} repetitions of {args.steps} steps"},
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "ms_per_step_reps": head["ms_per_step_reps"],
        "finite": head["finite"],
    }
    if not args.no_secondary and not two_d:
        other = "fp32" if args.precision == "fp64" else "fp64"
        sec = measure_line(args, wl, wkey, other, False, args.mesh)
        out["fp32_mixed" if other == "fp32" else "fp64"] = sec
        f32 = sec if other == "fp32" else head
        f64 = head if other == "fp32" else sec
        out["fp32_over_fp64"] = f32["value"] / f64["value"]
        if args.workload != "c2" and args.mesh == "equal":
            out["c2_fp64"] = measure_line(args, inputs.workload("c2"), "c2", "fp64", False, "equal")
        if args.workload == "c5" and args.mesh == "equal":
            # the other grids and meshes of the path, FP64, so that one run reports them all
            out["c3_fp64"] = measure_line(args, inputs.workload("c3"), "c3", "fp64", False, "equal")
            out["c2_graded_fp64"] = measure_line(args, inputs.workload("c2"), "c2-graded", "fp64", False, "graded")
            out["c2_distorted_fp64"] = measure_line(args, inputs.workload("c2"), "c2-distorted", "fp64", False,
                                                    "distorted")
            out["riemann_fp64"] = measure_line(args, workload_2d("riemann"), "riemann", "fp64", True, "equal")
    if args.adjoint_workload != "none" and not two_d:
        aover = {} if args.adjoint_cfl is None else {"cfl": args.adjoint_cfl}
        if args.adjoint_steps is not None:
            aover["steps"] = args.adjoint_steps
        wa = inputs.workload(args.adjoint_workload, **aover)
        out["adjoint"] = run_adjoint(wa, 0 if wa["precision"] == "fp64" else 1, mesh=args.mesh)
    if not args.no_cpu_baseline and args.mesh != "distorted":
        if two_d:
            out["cpu_baseline"] = cpu_baseline_2d(wl, args.cpu_budget)
        else:
            # the oracle on the 16^3-cell subcase of the same workload (same Ma, Re, CFL)
            sub = wl if wl["n_el"] <= 16 else inputs.workload(args.workload, n_el=16, **over)
            out["cpu_baseline"] = cpu_baseline(sub, args.cpu_budget, graded=args.mesh == "graded")
            if sub is not wl:
                out["cpu_baseline"]["sample"] += f" (the 16^3-cell subcase of the {wl['n_el']}^3-cell grid)"
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
