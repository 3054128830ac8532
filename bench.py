"""Throughput of the 2SHOC-RK4 integrator on the 2D Gross-Pitaevskii workload.

Workload: a = 0.5, s = -1, V = 0.5 (0.05)^2 r^2 on [-40, 40]^2, 2048 intervals per axis
(2049^2 nodes, 2047^2 interior points), Dirichlet 0, vortex in a Thomas-Fermi cloud
plus 1e-3 seeded complex noise; dt = 0.5 x the stability bound (4.0415e-4).  One
"step" is one classic RK4 step over the whole grid, with the kernel variant the
library's autotuner picks (the whole-step kernel: one launch per step).  Inputs are
resident in HBM before the timed region; K steps are timed with HIP events on the
solver's stream, bracketed by device synchronisation.

Prints one JSON line.  value = interior points x RK4 steps / s / 1e9 (FP64 path).
roofline: the dominant kernel's algorithmic work per launch / its mean launch time.
The whole-step kernel is bound by vector-ALU issue: achieved = 190 real flops per
interior point and step (FMA = 2) / launch time, against the vector peak of its type.
The four-launch stage kernels are timed beside it ("stage_kernels") with their HBM
roofline (76 B per interior point and launch for complex128).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import bench_traffic  # noqa: E402

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per interior point and RK4 step of the stage kernels (4 launches, V stored):
#   complex128 17*16 + 4*8 = 304; complex64 17*8 + 4*4 = 152; mixed (complex128 master) 192
BYTES_PER_POINT_STEP = {"f64": 304, "f32": 152, "mixed": 192}
# ... and of the whole-step kernel: Psi^n and V read, Psi^{n+1} written
WHOLE_STEP_BYTES = {"f64": 40, "f32": 20, "mixed": 36}
# ... and of the 3D two-stage kernels (two launches per step): stages 1+2 read Psi^n, V and write
# K, B; stages 3+4 read B, K, Psi^n, V and write Psi^{n+1} (f32: 28 + 36; mixed 36 + 52; f64 56 + 72)
PAIR3D_BYTES = {"f64": 128, "f32": 64, "mixed": 88}
# real flops of one RK4 step per interior point (FMA = 2): 4 x 41 for the two step-1
# differences, step 2 and F, plus 26 for the K_tot and Psi updates
FLOPS_PER_POINT_STEP = 190
# ... and in 1D: 4 x 27 (one step-1 difference 8, step 2 8, F 11) + 26
FLOPS_PER_POINT_STEP_1D = 134
VECTOR_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "mixed": 157.3}

METRIC = "2SHOC-RK4 Gpt·steps/s + % HBM peak; coarse+learned vs plain fine at equal L2 err"
# timed runs of at most this many steps are checked live against the oracle (cpu_baseline leg)
LIVE_CHECK_MAX_STEPS = 50


def measured_traffic(kind, prec, variant):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on this
    kernel variant and the kernel's sources have not changed since."""
    try:
        t = json.load(open(bench_traffic.traffic_file(kind)))
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != bench_traffic.source_sha(kind):
        return None
    ent = t.get("per_launch_bytes", {}).get(prec)
    if not ent or ent.get("variant") != variant:
        return None
    return ent["bytes"]


def measured_valu_issue(prec, variant):
    """VALU issue fraction of the whole-step kernel from the committed counter run, if it was taken
    on this variant and the kernel's sources have not changed since."""
    try:
        t = json.load(open(bench_traffic.valu_file()))
    except (OSError, ValueError):
        return None
    ent = t.get("per_launch", {}).get(prec)
    if t.get("source_sha") != bench_traffic.source_sha("step2d") or not ent or ent.get("variant") != variant:
        return None
    return ent["valu_issue"]


def parse_variants(spec):
    """"f64:6,f32:3" -> {"f64": 6, "f32": 3}; "" -> {}."""
    out = {}
    for item in filter(None, spec.split(",")):
        k, v = item.split(":")
        out[k] = int(v)
    return out


def time_solver(P, spec, prec, steps, warmup, variant=None, stencil=None, dt=None, check=None, settle_ms=100.0):
    """Time `steps` RK4 steps after `warmup` untimed ones; HIP events on the solver's stream.
    variant None: the library's autotuner picks the kernel variant (untimed).  With `check`, the
    timed steps start again from the initial field and check(final field) is returned as well.

    Before the warm-up steps, untimed steps keep the GPU busy for about `settle_ms`: a short timed
    window that starts after host-side idle time lands in the GPU's clock ramp (20-step windows
    measured up to 25 % slower than the 2000-step rate of the same kernel).  For the same reason the
    initial field of a `check` run is restored from a device copy, not from host memory."""
    import torch
    s = P.Solver.from_spec(spec, prec=prec)
    if stencil:
        s.stencil = stencil
    s.set_field(spec.psi0)
    psi0_dev = None
    if check is not None:
        psi0_dev = torch.from_numpy(np.ascontiguousarray(spec.psi0, dtype=s.dtype)).to("cuda")
    if dt is None:
        dt = 0.5 * s.max_dt()
    if variant is None:
        variant = s.autotune(reps=100)   # 2 x 100 steps of every variant: stable choice
    else:
        s.variant = variant
    stream = torch.cuda.current_stream()
    if settle_ms > 0:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(10, dt)
        e1.record(stream)
        torch.cuda.synchronize()
        s.step(int(settle_ms / max(e0.elapsed_time(e1) / 10, 1e-3)), dt)
    s.step(warmup, dt)
    if check is not None:
        s.set_field(psi0_dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    mass = s.mass()
    launches = s.launches_per_step() * steps
    checked = check(s.get_field()) if check is not None else None
    s.close()
    if check is not None:
        return ms, wall, launches, dt, mass, variant, checked
    return ms, wall, launches, dt, mass, variant


def best_stage_variant(P, spec, prec, steps=100):
    """Fastest of the four-launch stage-kernel variants (for the stage-kernel comparison)."""
    s = P.Solver.from_spec(spec, prec=prec)
    cands = []
    for v in range(s.variant_count()):
        s.variant = v
        if s.launches_per_step() == 4:
            cands.append(v)
    s.close()
    best = None
    for v in cands:
        ms = time_solver(P, spec, prec, steps, 5, variant=v)[0]
        if best is None or ms < best[0]:
            best = (ms, v)
    return best[1]


def copy_ceiling_gbs():
    """Achieved GB/s of a plain device copy of 1 GiB (read + write), for context."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 10 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_baseline(spec, budget_s=12.0, budget_1core_s=6.0, match_steps=None, dt=None):
    """The FP64 oracle on the same grid, a bounded number of RK4 steps on the host cores
    (all of them, then one).  With match_steps (at most 50), the all-cores run takes exactly that
    many steps from the initial field at step dt, the GPU's timed run, and its final field is
    returned too (the accuracy reference of that run)."""
    import oracle
    P = oracle.Problem.from_spec(spec)
    if dt is None:
        dt = 0.5 * P.max_dt(spec.psi0)

    def run(budget, cap):
        psi, steps, t0 = spec.psi0, 0, time.perf_counter()
        while True:
            psi = P.rk4(psi, 1, dt)
            steps += 1
            el = time.perf_counter() - t0
            if (el >= budget and match_steps is None) or steps >= cap:
                return steps, el, psi

    cores = oracle.threads()
    steps, el, final = run(budget_s, match_steps or 50)
    oracle.set_threads(1)
    match, match_steps = match_steps, None
    try:
        steps1, el1, _ = run(budget_1core_s, 10)
    finally:
        oracle.set_threads(cores)
        match_steps = match
    # the 1D soliton (config 1) is small enough to run whole: its wall time beside the GPU's
    import nlse_inputs as I
    sp1 = I.config_soliton_1d(1024)
    P1 = oracle.Problem.from_spec(sp1)
    n1, dt1 = oracle.steps_for(sp1.t_end, P1.max_dt(sp1.psi0))
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        P1.rk4(sp1.psi0, n1, dt1)
        el_1d = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    same = " (from the initial field at the GPU's step size: the timed run's accuracy reference)" \
        if match_steps else ""
    out = {"value": spec.interior_points * steps / el / 1e9, "unit": "Gpt·steps/s",
           "cores": cores, "kind": "oracle",
           "sample": f"{steps} RK4 steps of the FP64 oracle on the full {spec.grid.n + 1}^2 grid{same} ({el:.1f} s, "
                     f"{cores} threads); {steps1} steps on 1 thread ({el1:.1f} s)",
           "single_core_value": spec.interior_points * steps1 / el1 / 1e9,
           "soliton1d_full_run_s_1thread": el_1d, "soliton1d_steps": n1}
    return (out, final) if match_steps else (out, None)


def cpu_baseline_3d(n3d, budget_s=15.0, cap=5):
    """The FP64 oracle on config 3's full grid: up to `cap` RK4 steps on all host threads."""
    import oracle
    import nlse_inputs as I
    spec = I.config_gp3d(n=n3d)
    P = oracle.Problem.from_spec(spec)
    dt = 0.5 * P.max_dt(spec.psi0)
    psi, steps, t0 = spec.psi0, 0, time.perf_counter()
    while True:
        psi = P.rk4(psi, 1, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= cap:
            break
    cores = oracle.threads()
    return {"value": spec.interior_points * steps / el / 1e9, "unit": "Gpt·steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} RK4 steps of the FP64 oracle on the full {n3d + 1}^3 grid ({el:.1f} s, {cores} threads)"}


def cpu_baseline_batch(steps=10, every1d=16, every2d=8):
    """The FP64 oracle on a fixed sample of the batched workload's instances (every 16th 1D and
    every 8th 2D instance), `steps` RK4 steps each at 0.5 x its own bound, one after another."""
    import oracle
    import nlse_inputs as I
    specs = I.batch_instances()
    sample = [sp for i, sp in enumerate(specs) if sp.dim == 1 and i % every1d == 0]
    sample += [sp for i, sp in enumerate(x for x in specs if x.dim == 2) if i % every2d == 0]
    runs = []
    for sp in sample:
        P = oracle.Problem.from_spec(sp)
        runs.append((P, sp.psi0, 0.5 * P.max_dt(sp.psi0), sp.interior_points))
    t0 = time.perf_counter()
    for P, psi0, dt, _ in runs:
        P.rk4(psi0, steps, dt)
    el = time.perf_counter() - t0
    pts = sum(r[3] for r in runs) * steps
    n1 = sum(1 for sp in sample if sp.dim == 1)
    return {"value": pts / el / 1e9, "unit": "Gpt·steps/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{n1} 1D + {len(sample) - n1} 2D instances of the batched workload (every {every1d}th / "
                      f"{every2d}th), {steps} RK4 steps each ({el:.1f} s, {oracle.threads()} threads)"}


def bench_1d(P, I):
    """Config 1 (1D bright soliton, 1025 nodes, to t = 10): one launch of the on-chip solver for
    the whole run; wall time and the distance to the exact solution."""
    import torch
    sp = I.config_soliton_1d(1024)
    (x,) = sp.grid.coords()
    exact = I.bright_soliton(x, sp.t_end, 1.0, 1.0, 1.0, 0.5)
    res = {"workload": "1D bright soliton, 1025 nodes, a = s = 1, t = 10, dt = 0.5 k_max (config 1)"}
    for prec in ("f64", "f32"):
        for st in ("2shoc", "noncompact", "cd"):   # Sec. 5's comparison in 1D (on chip: latency, not bytes)
            s = P.Solver.from_spec(sp, prec=prec)
            s.stencil = st
            s.set_field(sp.psi0)
            variant = s.autotune(reps=8)   # workgroup size / node bound of the on-chip solver (untimed)
            nsteps = int(math.ceil(sp.t_end / (0.5 * s.max_dt())))
            dt = sp.t_end / nsteps
            s.step(10, dt)   # warm-up (discarded)
            s.set_field(sp.psi0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            s.step(nsteps, dt)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            g = np.asarray(s.get_field(), np.complex128)
            s.close()
            err = float(np.linalg.norm(g - exact) / np.linalg.norm(exact))
            r = {"steps": nsteps, "run_ms": ms, "us_per_step": 1e3 * ms / nsteps, "rel_l2_vs_exact": err,
                 "launches": 1, "solver_variant": variant}
            if st == "2shoc":
                res[prec] = r
            else:
                res[prec].setdefault("stencils", {})[st] = r
            print(f"[bench] 1D soliton {prec} {st}: {nsteps} steps in {ms:.2f} ms ({1e3 * ms / nsteps:.2f} us/step), "
                  f"rel L2 vs exact {err:.3e}", file=sys.stderr, flush=True)
    return res


def bench_3d(P, I, args):
    """The 3D Gross-Pitaevskii workload (HBM-resident working set of ~5 GB at 513^3)."""
    spec = I.config_gp3d(n=args.n3d)
    npts = spec.interior_points
    res = {"workload": f"3D Gross-Pitaevskii 2SHOC-RK4, {args.n3d + 1}^3 nodes, a=0.5 s=-1 omega=0.1 on "
                       "[-24,24]^3, Dirichlet 0, Thomas-Fermi cloud x vortex-ring phase",
           "interior_points": npts, "steps": args.steps3d}
    force3d = parse_variants(args.variant3d)
    # config 3's full run (500 steps) has a stored FP64 oracle state sampled at 1241 nodes
    # (tests/golden/gp3d_512_500steps.json, written by the oracle alone)
    gold = None
    gpath = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "gp3d_512_500steps.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)
        if gold["n"] != args.n3d:
            gold = None
    for prec in args.precs3d.split(","):
        ms, wall, launches, dt, mass, variant = time_solver(P, spec, prec, args.steps3d, 5, variant=force3d.get(prec))
        gpts = npts * args.steps3d / (ms * 1e-3) / 1e9
        lps = launches // args.steps3d
        pairs = lps == 2   # the autotuner picked the two-stage kernels
        step_bytes = (PAIR3D_BYTES if pairs else BYTES_PER_POINT_STEP)[prec] * npts
        per_launch_bytes = step_bytes / lps
        achieved = per_launch_bytes / (ms * 1e-3 / launches) / 1e9
        stage_eq = BYTES_PER_POINT_STEP[prec] * npts * args.steps3d / (ms * 1e-3) / 1e9
        res[prec] = {"value": gpts, "unit": "Gpt·steps/s", "ms_per_step": ms / args.steps3d, "dt": dt,
                     "launches_per_step": lps,
                     "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": achieved / HBM_PEAK_GBS,
                                  "traffic": measured_traffic("pair3d", prec, variant) if pairs else None,
                                  "kernel": "nlse::pair3d_kernel" if pairs else "nlse::stage3d_kernel",
                                  "algorithmic_bytes_per_launch": per_launch_bytes,
                                  "stage_equivalent_gbs": stage_eq, "stage_equivalent_frac": stage_eq / HBM_PEAK_GBS,
                                  "avg_launch_us": ms * 1e3 / launches, "tile_variant": variant}}
        if gold is not None:   # the full run again from the initial field, outside any timed region
            s = P.Solver.from_spec(spec, prec=prec)
            s.set_field(spec.psi0)
            s.variant = variant
            s.step(gold["steps"], gold["dt"])
            iz, iy, ix = np.array(gold["nodes"]).T
            ref = np.array(gold["re"]) + 1j * np.array(gold["im"])
            got = np.asarray(s.get_field())[iz, iy, ix].astype(np.complex128)
            s.close()
            res[prec]["rel_l2_vs_fp64_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            res[prec]["accuracy_check"] = ("sampled relative L2 (1241 nodes) against the stored FP64 oracle "
                                           f"state after the full {gold['steps']}-step run")
        print(f"[bench] 3D {prec}: {gpts:.2f} Gpt*steps/s, {ms / args.steps3d:.3f} ms/step, {lps} launches/step, "
              f"{achieved:.0f} GB/s algorithmic ({100 * achieved / HBM_PEAK_GBS:.1f}% of HBM peak; "
              f"{stage_eq:.0f} GB/s in the four-launch form's bytes)", file=sys.stderr, flush=True)
        if "rel_l2_vs_fp64_oracle" in res[prec]:
            print(f"[bench] 3D {prec} full {gold['steps']}-step run: rel L2 vs FP64 oracle "
                  f"{res[prec]['rel_l2_vs_fp64_oracle']:.2e}", file=sys.stderr, flush=True)
        if pairs and not args.no_stage3d:   # the four-launch stage kernels on the same workload, for comparison
            sv = min(range(4), key=lambda v: time_solver(P, spec, prec, 20, 2, variant=v)[0])
            ms_s, _, launches_s, _, _, _ = time_solver(P, spec, prec, args.steps3d, 5, variant=sv)
            ach_s = BYTES_PER_POINT_STEP[prec] * npts * args.steps3d / (ms_s * 1e-3) / 1e9
            res[prec]["stage_kernels"] = {"value": npts * args.steps3d / (ms_s * 1e-3) / 1e9,
                                          "ms_per_step": ms_s / args.steps3d, "tile_variant": sv,
                                          "roofline": {"bound": "hbm", "achieved": ach_s, "peak": HBM_PEAK_GBS,
                                                       "unit": "GB/s", "frac": ach_s / HBM_PEAK_GBS,
                                                       "kernel": "nlse::stage3d_kernel"}}
            print(f"[bench] 3D {prec} stage kernels: {res[prec]['stage_kernels']['value']:.2f} Gpt*steps/s, "
                  f"{ach_s:.0f} GB/s algorithmic ({100 * ach_s / HBM_PEAK_GBS:.1f}% of HBM peak)",
                  file=sys.stderr, flush=True)
        if not args.no_stencils:   # Sec. 5's comparison in 3D: stage kernels, same bytes per point-step
            sv3 = res[prec]["stage_kernels"]["tile_variant"] if "stage_kernels" in res[prec] else \
                (0 if pairs else variant)
            steps_x = max(args.steps3d // 4, 1)
            for st in ("2shoc", "noncompact", "cd"):
                ms_x = time_solver(P, spec, prec, steps_x, 3, variant=sv3, stencil=st)[0]
                bw = BYTES_PER_POINT_STEP[prec] * npts * steps_x / (ms_x * 1e-3) / 1e9
                res[prec].setdefault("stencils_stage_kernels", {})[st] = {
                    "value": npts * steps_x / (ms_x * 1e-3) / 1e9, "ms_per_step": ms_x / steps_x,
                    "algorithmic_gbs": bw, "hbm_frac": bw / HBM_PEAK_GBS, "tile_variant": sv3}
                print(f"[bench] 3D stencil {st} {prec} (stage kernels): "
                      f"{npts * steps_x / (ms_x * 1e-3) / 1e9:.2f} Gpt*steps/s, {100 * bw / HBM_PEAK_GBS:.1f}% of HBM peak",
                      file=sys.stderr, flush=True)
    return res


def bench_batch(P, I, steps=1000):
    """The batched workload: 4096 1D instances (n ~ U[256, 8192], bright / dark solitons) and
    256 2D GP instances at 256^2 (omega ~ U[0.02, 0.1]), complex64, one graph launch of
    `steps` RK4 steps for every instance."""
    import torch
    specs = I.batch_instances()
    b = P.Batch(specs, prec="f32")
    b.set_fields(specs)
    b.set_dts(0.5)
    variant = b.autotune(nsteps=50)
    # the autotuner's margin: 50 steps of each variant again, best of three (untimed region)
    tune = {}
    for v in range(b.variant_count()):
        b.variant = v
        b.step(50)   # graph capture for this variant
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            b.step(50)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            best = min(best or 1e30, e0.elapsed_time(e1))
        tune[v] = best
    b.variant = variant
    b.set_fields(specs)   # the timed run starts from the initial fields again
    pts1 = sum((sp.grid.n - 1) for sp in specs if sp.dim == 1)
    pts2 = sum((sp.grid.n - 1) ** 2 for sp in specs if sp.dim == 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(torch.cuda.current_stream())
    b.step(steps)
    e1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    gpts = (pts1 + pts2) * steps / (ms * 1e-3) / 1e9
    flops = (FLOPS_PER_POINT_STEP * pts2 + FLOPS_PER_POINT_STEP_1D * pts1) * steps
    tflops = flops / (ms * 1e-3) / 1e12
    # HBM: a 2D instance reads Psi^n and V and writes Psi^{n+1} per step (whole-step kernel);
    # a 1D instance reads and writes its field once per launch (it lives on chip in between)
    hbm = WHOLE_STEP_BYTES["f32"] * pts2 * steps / (ms * 1e-3) / 1e9
    b.close()
    print(f"[bench] batch: {gpts:.2f} Gpt*steps/s over {len(specs)} instances, {ms:.1f} ms for {steps} steps",
          file=sys.stderr, flush=True)
    return {"workload": "4096 1D NLSE (n in [256, 8192], s = +-1, bright Dirichlet / dark MSD) + 256 2D GP "
                        "at 256^2 (omega in [0.02, 0.1]), complex64, one persistent graph launch",
            "instances": len(specs), "steps": steps, "interior_point_steps": (pts1 + pts2) * steps,
            "value": gpts, "unit": "Gpt·steps/s", "ms": ms, "tile_variant": variant,
            "autotune_ms_per_50_steps": tune,
            "autotune_margin": sorted(tune.values())[1] / sorted(tune.values())[0] - 1.0 if len(tune) > 1 else None,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": VECTOR_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                         "frac": tflops / VECTOR_PEAK_TFLOPS["f32"], "traffic": None,
                         "kernel": "nlse::batch2d_kernel + nlse::batch1d_kernel (one graph launch)",
                         "algorithmic_flops": flops,
                         "flops_per_point_step": {"2d": FLOPS_PER_POINT_STEP, "1d": FLOPS_PER_POINT_STEP_1D},
                         "attainable_peak_without_packed_fp32": VECTOR_PEAK_TFLOPS["f64"],
                         "hbm_gbs_algorithmic": hbm, "hbm_frac_algorithmic": hbm / HBM_PEAK_GBS}}


def bench_msd(P, I, args, res, npts):
    """2D MSD boundary (Sec. 3.2, extended to 2D): vortex-antivortex pairs in a uniform background,
    V = 0, on the 2049^2 grid; stage kernels plus the boundary launch before each stage, against the
    Dirichlet stage kernels of the same tile variant; and the autotuned MSD path (a whole-step
    kernel that forms the boundary itself) against the Dirichlet whole-step kernel."""
    g = I.grid(2, args.n, -80.0, 80.0)
    spec = I.ProblemSpec("msd2d", g, 0.5, -1.0, None, I.background_vortices(g, pairs=4, seed=3), "msd")
    out = {"workload": f"2D NLSE with the MSD boundary, {args.n + 1}^2 nodes, a=0.5 s=-1 V=0 on [-80,80]^2, "
                       "4 vortex-antivortex pairs in a uniform background + 1e-3 noise",
           "interior_points": npts}
    steps = max(args.steps // 4, 100)   # at least 100 steps: a few-step window is mostly launch latency
    for prec in ("f64", "f32"):
        if prec not in res:
            continue
        sv = res[prec]["stage_kernels"]["roofline"]["tile_variant"]
        ms, _, launches, dt, _, _ = time_solver(P, spec, prec, steps, 10, variant=sv)
        gpts = npts * steps / (ms * 1e-3) / 1e9
        ref = res[prec]["stage_kernels"]["ms_per_step"]
        out[prec] = {"value": gpts, "unit": "Gpt·steps/s", "ms_per_step": ms / steps, "dt": dt,
                     "launches_per_step": launches // steps, "tile_variant": sv,
                     "dirichlet_stage_ms_per_step": ref, "boundary_overhead": ms / steps / ref - 1.0}
        print(f"[bench] MSD 2D {prec} (stage kernels + boundary launches): {gpts:.2f} Gpt*steps/s, "
              f"{100 * out[prec]['boundary_overhead']:.1f}% over Dirichlet", file=sys.stderr, flush=True)
        ms, _, launches, dt, _, v = time_solver(P, spec, prec, steps, 10)
        gw = npts * steps / (ms * 1e-3) / 1e9
        refw = res[prec]["ms_per_step"]
        out[prec]["autotuned"] = {"value": gw, "unit": "Gpt·steps/s", "ms_per_step": ms / steps,
                                  "launches_per_step": launches // steps, "tile_variant": v,
                                  "dirichlet_whole_step_ms_per_step": refw,
                                  "overhead_vs_dirichlet_whole_step": ms / steps / refw - 1.0}
        print(f"[bench] MSD 2D {prec} autotuned (variant {v}, {launches // steps} launch/step): {gw:.2f} "
              f"Gpt*steps/s, {100 * (ms / steps / refw - 1.0):.1f}% over the Dirichlet whole step",
              file=sys.stderr, flush=True)
    return out


def bench_msd3d(P, I, args, res3d):
    """3D MSD boundary: a vortex ring of radius 8 in a uniform background, V = 0, on the 513^3 grid
    of config 3 ([-24, 24]^3); stage kernels plus the boundary launch before each stage (1.6 M
    boundary nodes), against the Dirichlet stage kernels of config 3 with the same tile variant."""
    g = I.grid(3, args.n3d, -24.0, 24.0)
    spec = I.ProblemSpec("msd3d", g, 0.5, -1.0, None, I.background_ring(g, ring_radius=8.0), "msd")
    npts = spec.interior_points
    out = {"workload": f"3D NLSE with the MSD boundary, {args.n3d + 1}^3 nodes, a=0.5 s=-1 V=0 on [-24,24]^3, "
                       "a vortex ring of radius 8 in a uniform background", "interior_points": npts}
    steps = max(args.steps3d // 4, 1)
    for prec in ("f32",):
        r = res3d.get(prec, {})
        if "stage_kernels" not in r:
            continue
        sv = r["stage_kernels"]["tile_variant"]
        ms, _, launches, dt, _, _ = time_solver(P, spec, prec, steps, 3, variant=sv)
        gpts = npts * steps / (ms * 1e-3) / 1e9
        ref = r["stage_kernels"]["ms_per_step"]
        out[prec] = {"value": gpts, "unit": "Gpt·steps/s", "ms_per_step": ms / steps, "dt": dt,
                     "launches_per_step": launches // steps, "tile_variant": sv,
                     "dirichlet_stage_ms_per_step": ref, "boundary_overhead": ms / steps / ref - 1.0}
        print(f"[bench] MSD 3D {prec} (stage kernels + boundary launches): {gpts:.2f} Gpt*steps/s, "
              f"{100 * out[prec]['boundary_overhead']:.1f}% over Dirichlet", file=sys.stderr, flush=True)
    return out


def bench_learned(P, seeds=(9000, 9001, 9002, 9003)):
    """Coarse (513^2) + learned corrector vs plain runs, all against the FP64 2049^2 plain run at
    t = 20, on the four held-out seeds with the committed weights (trained on the GPU by the
    library's kernels); mean errors, the worst seed's gain and the equal-error speedup."""
    from paper_1109_1027_amd import corrector as K
    params, scale = K.load_weights()
    res = K.evaluate(params, scale, list(seeds))
    summ = K.summarize(res)
    print(f"[bench] learned ({len(seeds)} held-out seeds): E_plain(513^2) {summ['E_plain'][512]:.3e}, "
          f"E_learned {summ['E_learned']:.3e}, mean gain {summ['gain_E512_over_learned']:.2f}x (worst "
          f"{summ['gain_worst']:.2f}x), equal-error speedup {summ['speedup_vs_plain_equal_error']:.2f}x",
          file=sys.stderr, flush=True)
    return {"metric": "coarse+learned vs plain at equal L2 error (vs the FP64 2049^2 plain run, t = 20)",
            "workload": "2D GP, a=0.5 s=-1 omega=0.05, 1-8 vortices + 1e-3 noise, held-out seeds 9000-9003; "
                        "coarse 513^2 with the 3-layer BF16-MFMA conv corrector every 10 steps",
            **{k: summ[k] for k in ("seeds", "E_plain", "T_plain_s", "E_learned", "T_learned_s", "T_fine_s",
                                    "fit_order_p", "n_equal_error", "speedup_vs_plain_equal_error",
                                    "speedup_vs_fine", "gain_E512_over_learned", "gain_per_seed", "gain_worst",
                                    "E_fine_run_richardson")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048, help="intervals per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precs", default="f64,f32,mixed")
    ap.add_argument("--n3d", type=int, default=512, help="intervals per axis of the 3D workload (0: skip)")
    ap.add_argument("--precs3d", default="f32,mixed")
    ap.add_argument("--steps3d", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=1000, help="steps of the batched workload (0: skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-corrector comparison")
    ap.add_argument("--no-stencils", action="store_true", help="skip the 2SHOC / non-compact / CD comparison")
    ap.add_argument("--no-msd", action="store_true", help="skip the 2D MSD-boundary measurement")
    ap.add_argument("--variant2d", default="", help="force 2D kernel variants per precision, e.g. f64:6,f32:3 "
                                                    "(default: the library's autotuner)")
    ap.add_argument("--stage-variant", default="", help="force the stage-kernel comparison variants, e.g. f64:1")
    ap.add_argument("--variant3d", default="", help="force 3D kernel variants per precision, e.g. f32:4,mixed:5")
    ap.add_argument("--no-stage3d", action="store_true", help="skip the 3D stage-kernel comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(instances of the solver shard by domain slabs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import nlse_inputs as I
    import paper_1109_1027_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.load()
    spec = I.config_gp2d(n=args.n)
    npts = spec.interior_points
    precs = args.precs.split(",")
    force2d, force_stage = parse_variants(args.variant2d), parse_variants(args.stage_variant)
    res = {}
    # The full benchmark run (2000 steps at 2049^2) has a stored FP64 oracle state, sampled at 545
    # nodes (tests/golden/gp2d_2048_2000steps.json, written by the oracle alone): each precision's
    # timed run starts from the initial field with the oracle's dt and is compared with it.
    # Other step counts up to 50 (the driver's short run among them) keep their final fields and
    # are compared over every node with the FP64 oracle's run of the same steps in the
    # cpu_baseline leg below.
    golden, check, gold_dt = None, None, None
    gpath = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "gp2d_2048_2000steps.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            golden = json.load(f)
        if golden["n"] != args.n:
            golden = None
        else:
            gold_dt = golden["dt"]   # the oracle's step size on this grid (0.5 x its bound)
            if golden["steps"] != args.steps:
                golden = None
    live = golden is None and args.steps <= LIVE_CHECK_MAX_STEPS and not args.no_cpu_baseline
    if golden is not None:
        iy, ix = np.array(golden["nodes"]).T
        gref = np.array(golden["re"]) + 1j * np.array(golden["im"])

        def check(field):
            got = np.asarray(field, np.complex128)[iy, ix]
            return float(np.linalg.norm(got - gref) / np.linalg.norm(gref))
    elif live:
        def check(field):
            return np.array(field, np.complex128)
    finals = {}
    for prec in precs:
        timed = time_solver(P, spec, prec, args.steps, args.warmup, variant=force2d.get(prec),
                            dt=gold_dt, check=check)
        ms, wall, launches, dt, mass, variant = timed[:6]
        err = timed[6] if len(timed) > 6 else None
        if live:
            finals[prec], err = err, None
        gpts = npts * args.steps / (ms * 1e-3) / 1e9
        avg_launch_s = ms * 1e-3 / launches
        whole = launches == args.steps
        if whole:
            flops = FLOPS_PER_POINT_STEP * npts
            bytes_ = WHOLE_STEP_BYTES[prec] * npts
            achieved = flops / avg_launch_s / 1e12
            roof = {"bound": "alu", "achieved": achieved, "peak": VECTOR_PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                    "frac": achieved / VECTOR_PEAK_TFLOPS[prec], "traffic": measured_traffic("step2d", prec, variant),
                    "kernel": "nlse::step2d_kernel", "algorithmic_flops_per_launch": flops,
                    "algorithmic_bytes_per_launch": bytes_, "hbm_gbs_algorithmic": bytes_ / avg_launch_s / 1e9,
                    "hbm_frac_algorithmic": bytes_ / avg_launch_s / 1e9 / HBM_PEAK_GBS,
                    "valu_issue_measured": measured_valu_issue(prec, variant),
                    "stage_equivalent_gbs": BYTES_PER_POINT_STEP[prec] * npts / avg_launch_s / 1e9,
                    "avg_launch_us": avg_launch_s * 1e6, "tile_variant": variant}
            if prec != "f64":
                roof["attainable_peak_without_packed_fp32"] = VECTOR_PEAK_TFLOPS["f64"]
            note = (f"{achieved:.2f} TFLOP/s algorithmic ({100 * roof['frac']:.1f}% of the {prec} vector peak), "
                    f"{roof['hbm_gbs_algorithmic']:.0f} GB/s of HBM")
        else:
            bytes_ = BYTES_PER_POINT_STEP[prec] * npts / 4
            achieved = bytes_ / avg_launch_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("stage2d", prec, variant),
                    "kernel": "nlse::stage2d_kernel", "algorithmic_bytes_per_launch": bytes_,
                    "avg_launch_us": avg_launch_s * 1e6, "tile_variant": variant}
            note = f"{achieved:.0f} GB/s algorithmic ({100 * roof['frac']:.1f}% of HBM peak)"
        res[prec] = {"value": gpts, "ms_per_step": ms / args.steps, "wall_s": wall, "dt": dt, "mass_end": mass,
                     "launches_per_step": launches // args.steps, "roofline": roof,
                     "rel_l2_vs_fp64_oracle": err,
                     "accuracy_check": ("sampled relative L2 (545 nodes) against the stored FP64 oracle state "
                                        "after the same 2000 steps" if err is not None else None)}
        if err is not None:
            note += f", rel L2 vs FP64 oracle {err:.2e}"
        print(f"[bench] {prec}: {gpts:.2f} Gpt*steps/s, {ms / args.steps:.4f} ms/step, {note}",
              file=sys.stderr, flush=True)
        # the four-launch stage kernels on the same workload, with their HBM roofline
        sv = force_stage[prec] if prec in force_stage else best_stage_variant(P, spec, prec)
        ms_s, _, launches_s, _, _, _ = time_solver(P, spec, prec, args.steps, args.warmup, variant=sv)
        per_launch = BYTES_PER_POINT_STEP[prec] * npts / 4
        avg_s = ms_s * 1e-3 / launches_s
        ach_s = per_launch / avg_s / 1e9
        res[prec]["stage_kernels"] = {
            "value": npts * args.steps / (ms_s * 1e-3) / 1e9, "ms_per_step": ms_s / args.steps,
            "roofline": {"bound": "hbm", "achieved": ach_s, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach_s / HBM_PEAK_GBS, "traffic": measured_traffic("stage2d", prec, sv),
                         "kernel": "nlse::stage2d_kernel", "algorithmic_bytes_per_launch": per_launch,
                         "avg_launch_us": avg_s * 1e6, "tile_variant": sv}}
        print(f"[bench] {prec} stage kernels: {res[prec]['stage_kernels']['value']:.2f} Gpt*steps/s, "
              f"{ach_s:.0f} GB/s algorithmic ({100 * ach_s / HBM_PEAK_GBS:.1f}% of HBM peak)",
              file=sys.stderr, flush=True)
    # Sec. 5's comparison on this hardware: the stage kernels with the 2SHOC, the non-compact
    # fourth-order and the second-order CD Laplacian (same bytes, different operation counts)
    stencils, stencils_ws = {}, {}
    if not args.no_stencils:
        for prec in ("f64", "f32"):
            if prec not in res:
                continue
            sv = res[prec]["stage_kernels"]["roofline"]["tile_variant"]
            for st in ("2shoc", "noncompact", "cd"):
                ms_s = time_solver(P, spec, prec, args.steps // 4, 10, variant=sv, stencil=st)[0]
                steps_s = args.steps // 4
                bw = BYTES_PER_POINT_STEP[prec] * npts * steps_s / (ms_s * 1e-3) / 1e9
                stencils.setdefault(prec, {})[st] = {"value": npts * steps_s / (ms_s * 1e-3) / 1e9,
                                                     "ms_per_step": ms_s / steps_s, "algorithmic_gbs": bw,
                                                     "hbm_frac": bw / HBM_PEAK_GBS, "tile_variant": sv}
                print(f"[bench] stencil {st} {prec} (stage kernels): {stencils[prec][st]['value']:.2f} Gpt*steps/s, "
                      f"{100 * bw / HBM_PEAK_GBS:.1f}% of HBM peak", file=sys.stderr, flush=True)
            # the same comparison in the whole-step kernel (one launch per step, vector-ALU bound),
            # where the stencils' operation counts show; variant chosen by the autotuner per stencil
            for st in ("2shoc", "noncompact", "cd"):
                steps_w = max(args.steps, 200)
                ms_w, _, launches_w, _, _, v_w = time_solver(P, spec, prec, steps_w, 10, stencil=st)
                stencils_ws.setdefault(prec, {})[st] = {
                    "value": npts * steps_w / (ms_w * 1e-3) / 1e9, "ms_per_step": ms_w / steps_w,
                    "launches_per_step": launches_w // steps_w, "tile_variant": v_w}
                print(f"[bench] stencil {st} {prec} (whole-step kernel): "
                      f"{stencils_ws[prec][st]['value']:.2f} Gpt*steps/s", file=sys.stderr, flush=True)
    main_prec = precs[0]
    out = {
        "metric": METRIC, "value": res[main_prec]["value"], "unit": "Gpt·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res[main_prec]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "mixed": "f32+f64"}[main_prec], "data": "synthetic",
        "config": {"workload": "2D Gross-Pitaevskii 2SHOC-RK4, 2049^2 nodes (2047^2 interior), "
                               "a=0.5 s=-1 omega=0.05 on [-40,40]^2, Dirichlet 0, vortex+1e-3 noise, "
                               f"dt=0.5*k_max={res[main_prec]['dt']:.6g}",
                   "grid_nodes": [args.n + 1, args.n + 1], "interior_points": npts,
                   "precision": main_prec, "parallelism": "single GPU"},
        "roofline": res[main_prec]["roofline"],
        "stage_kernels": res[main_prec]["stage_kernels"],
        "rel_l2_vs_fp64_oracle": res[main_prec]["rel_l2_vs_fp64_oracle"],
        "accuracy_check": res[main_prec]["accuracy_check"],
        "variants": {p: {k: v for k, v in r.items()
                         if k in ("value", "ms_per_step", "roofline", "stage_kernels", "rel_l2_vs_fp64_oracle")}
                     for p, r in res.items() if p != main_prec},
    }
    try:
        out["copy_ceiling_gbs"] = copy_ceiling_gbs()
    except Exception as e:  # context only
        out["copy_ceiling_gbs"] = None
        print(f"[bench] copy ceiling failed: {e}", file=sys.stderr)
    if stencils:
        out["stencils_stage_kernels"] = stencils
    if stencils_ws:
        out["stencils_whole_step"] = stencils_ws
    if not args.no_msd:
        out["msd2d"] = bench_msd(P, I, args, res, npts)
    out["soliton1d"] = bench_1d(P, I)
    if args.n3d > 0:
        out["gp3d"] = bench_3d(P, I, args)
        if not args.no_msd and not args.no_stage3d:
            out["msd3d"] = bench_msd3d(P, I, args, out["gp3d"])
    if args.batch_steps > 0:
        out["batch"] = bench_batch(P, I, args.batch_steps)
    if not args.no_learned:
        out["learned"] = bench_learned(P)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        out["cpu_baseline"], ref = cpu_baseline(spec, match_steps=args.steps if live else None,
                                                dt=res[main_prec]["dt"] if live else None)
        if ref is not None:   # accuracy of each timed run: every node against the oracle's same steps
            for prec, f in finals.items():
                e = float(np.linalg.norm((f - ref).ravel()) / np.linalg.norm(ref.ravel()))
                tgt = out if prec == main_prec else out["variants"][prec]
                tgt["rel_l2_vs_fp64_oracle"] = e
                if prec == main_prec:
                    out["accuracy_check"] = (f"relative L2 over all {ref.size} nodes against the FP64 oracle's run "
                                             f"of the same {args.steps} steps from the same initial field and dt")
                print(f"[bench] {prec}: rel L2 vs FP64 oracle after the timed {args.steps} steps {e:.2e}",
                      file=sys.stderr, flush=True)
        if args.n3d > 0:
            out["cpu_baseline"]["gp3d"] = cpu_baseline_3d(args.n3d)
        if args.batch_steps > 0:
            out["cpu_baseline"]["batch"] = cpu_baseline_batch()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
