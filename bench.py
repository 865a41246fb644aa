"""Benchmark of the explicit residual evaluation on one MI355X.

Workload: periodic 64^3 hexahedral Taylor-Green vortex (262,144 cells) at
Mach 0.1, Navier-Stokes Re 1600, P2 CWENOZ reconstruction, HLLC, Green-Gauss
viscous gradients, SSP-RK3 at CFL 0.5, with the per-step kinetic-energy
reduction.  A step = dt + 3 x (reconstruct, gradients, face flux, residual +
RK stage) + KE, all through the C ABI on one stream; inputs already resident
in HBM when the timed region starts.  By default 200 timed steps after 5
warm-up steps from the initial state: the vortex develops troubled cells as
it runs, so the gated variant's rate depends on the window.

Prints one JSON line: the headline variant's cell-stage updates/s, both
variants (FP64 plain and FP32 reconstruction/flux), the roofline of the
dominant kernel (reconstruction) timed with HIP events on its launch stream
around each of its calls in a replay of the timed steps, and the FP64 CPU
oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The dominant step is the reconstruction: one ucns_reconstruct call, timed
# as a whole with HIP events; its kernels, and the record of their measured
# HBM bytes per call (rocprofv3 counters, summed over the call's kernels)
def recon_kernels(head, grad):
    """Kernel names of one reconstruction call (main pass | positivity pass);
    grad: the gradients the main pass also forms (0 none, 1 Green-Gauss,
    2 least squares)."""
    t, g = ("float", "true") if head == "fp32_gate" else ("double", "false")
    return f"reconstruct_kernel<{t}, 9, false, {g}, {grad}>|reconstruct_fallback_kernel<{t}, 9>"



TRAFFIC = {"fp32_gate": "traffic_reconstruct_fp32_gate_tgv64.md",
           "fp64_plain": "traffic_reconstruct_fp64_tgv64.md"}
METRIC = "cell-stage updates/s, P2 CWENO+HLLC: FP64 plain vs FP32+MLP gate; % HBM peak"


def recon_bytes_per_cell(lm, precision, linear=False, gate=False, grad=False):
    """Algorithmic HBM bytes of one reconstruction of one cell: every operator
    value and index read once (the basis at a face point is recomputed from
    the point's 3 scaled coordinates and the cell's K basis means; one byte
    per face slot gives its point count), the directional-stencil count, the
    cell's own state read once, its face-point states and flag written once
    (neighbour states are re-reads of resident data).  linear: the cell
    takes the central polynomial only (no directional operators or
    indices).  gate: the in-kernel network's per-cell inputs (face-neighbour
    ids and offsets, basis scale, stencil size) and its mask output.  grad:
    the call also forms the Green-Gauss gradients (the face-neighbour ids,
    unless the gate has read them, each face slot's three weights, the twelve
    gradient values written).  At order 4 the call also stages the state
    cell-interleaved (40 bytes read, 64 written per cell)."""
    t = 8 if precision == 0 else 4
    K, MC, MD, ND, NF, Q = lm.K, lm.mc_pad, max(1, lm.md_pad), max(1, lm.nd_max), lm.nfmax, lm.qmax
    KD = getattr(lm, "kd", 3)  # terms of a directional polynomial (3 linear, 9 quadratic at P4)
    ops = K * MC + NF * Q * 3 + K + (0 if linear else K * (K + 1) // 2 + ND * KD * MD)
    idx = MC + (0 if linear else ND * MD)
    extra = (4 * NF + 3 * NF * t + t + 1 + 1) if gate else 0
    stage = 40 + 64 if K == 34 else 0
    ggrad = ((0 if gate else 4 * NF) + 3 * NF * t + 12 * t) if grad else 0
    return t * ops + 4 * idx + NF + 1 + 40 + t * 5 * NF * Q + 1 + extra + stage + ggrad


def step_bytes_per_cell(lm, precision, viscous=True, recon=None, fused=False):
    """Algorithmic HBM bytes of one stage of the whole path per cell (recon:
    the reconstruction's share, default the full CWENOZ one; fused: the
    gradients are part of it)."""
    t = 8 if precision == 0 else 4
    faces_per_cell = lm.n_face / lm.n_cell
    Q, NF = lm.qmax, lm.nfmax
    recon = recon_bytes_per_cell(lm, precision) if recon is None else recon
    flux = faces_per_cell * (2 * Q * 5 * t + t * (7 + Q) + 9 + 5 * t + (24 * t if viscous else 0))
    grad = (40 + 4 * NF + 12 * t + faces_per_cell * (8 + 4 * t)) if viscous and not fused else 0
    resid = 4 * NF + 5 * t * NF + 8 + 40 * 3
    return recon + flux + grad + resid


def time_steps(solver, U, steps, warmup, torch, graph=False):
    """Wall time of `steps` steps after `warmup` untimed ones; with graph, the
    step is captured once (after the warm-up) and replayed."""
    for _ in range(warmup):
        solver.step(U, ke=True)
    if graph:
        solver.capture(U)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        if graph:
            solver.step_graph(U)
        else:
            solver.step(U, ke=True)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall


def time_recon_replay(solver, U0, steps, warmup, torch):
    """Mean duration (ms) of the reconstruction calls (all the kernels one
    call launches) of the timed steps, from HIP events recorded on the launch
    stream around each call, and the mean fraction of cells the network took
    as smooth in those calls (0 without the network).  The events would add
    gaps to the timed loop, so the warm-up and timed steps are replayed from
    the same initial state (the path is deterministic: the same states, the
    same troubled cells) with the events in place."""
    U = torch.tensor(U0, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        solver.step(U, ke=True)
    solver.recon_events = []
    for _ in range(steps):
        solver.step(U, ke=True)
    torch.cuda.synchronize()
    ev, solver.recon_events = solver.recon_events, None
    ms = sum(a.elapsed_time(b) for a, b, _ in ev) / len(ev)
    smooth = [float(n) for _, _, n in ev if n is not None]
    frac = sum(smooth) / (len(smooth) * solver.mesh.n_cell) if smooth else 0.0
    return ms, frac


def copy_calibration(torch, nbytes=256 << 20):
    """One plain device copy of known size (read nbytes, write nbytes) outside
    the timed region: the reference for the HBM byte counters."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    return nbytes


def _cpu_baseline_child(lib_path, threads):
    """Child process of cpu_baseline (no GPU): the tuned oracle on the 32^3
    TGV (mesh built on all `threads`), 3 timed runs of 30 SSP-RK3 steps on
    `threads` threads, then one run of 6 steps on 1 thread, each from the
    same initial state; prints one JSON line of cell-stage rates."""
    import ctypes

    os.environ["OMP_NUM_THREADS"] = str(threads)
    import oracle
    from paper_2609_07387_amd import inputs

    oracle.use_library(lib_path)
    gomp = ctypes.CDLL("libgomp.so.1")   # the OpenMP runtime the oracle runs on
    m = inputs.periodic_hex_mesh(32)
    U0 = inputs.tgv_initial(m)
    om = oracle.OracleMesh(m, order=2)
    ph = oracle.phys(flux="hllc", viscous=True)
    out = {}
    for name, nthr, steps, runs in (("all", threads, 30, 3), ("one", 1, 6, 1)):
        gomp.omp_set_num_threads(nthr)
        rates = []
        for _ in range(runs):
            t0 = time.perf_counter()
            om.run(U0, ph, 0.5, steps)
            rates.append(m.n_cell * 3 * steps / (time.perf_counter() - t0))
        out[name] = rates
    print(json.dumps(out), flush=True)


def _lscpu():
    import subprocess

    out = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        return out
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
            out[k.strip()] = v.strip()
    return out


def cpu_baseline():
    """The FP64 oracle, unchanged but built -O3 -march=native for this host,
    on the 32^3 hex TGV with the same scheme (per-cell work is that of the
    64^3 workload), mesh build excluded: the mean of 3 runs on the threads
    this process may use (OMP_NUM_THREADS, else its CPU affinity), and one
    run on 1 thread, in a child process (no GPU; about 30 s of host time)."""
    import subprocess
    import tempfile

    import oracle

    tmp = tempfile.mkdtemp(prefix="ucns_oracle_")
    lib_path = oracle.build(out=os.path.join(tmp, "liboracle_tuned.so"), tuned=True)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", lib_path, str(threads)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, env=dict(os.environ))
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed: {r.stderr[-2000:]}")
    legs = json.loads(r.stdout.strip().splitlines()[-1])
    mean = sum(legs["all"]) / len(legs["all"])
    cpu = _lscpu()
    return {"value": mean, "unit": "cell-stage updates/s", "cores": threads, "kind": "oracle",
            "sample": "32^3 periodic hex TGV, same scheme (P2 CWENOZ, HLLC, NS, Green-Gauss); mean of 3 runs of 30 "
                      "SSP-RK3 steps on the threads shown, plus 6 steps on 1 thread; oracle built -O3 "
                      "-march=native on this host; mesh build excluded",
            "runs": legs["all"], "spread": (max(legs["all"]) - min(legs["all"])) / mean,
            "one_thread": legs["one"][0], "host": cpu}


GRAD_NAME = {"green_gauss": "Green-Gauss", "least_squares": "least-squares"}
RK_NAME = {"ssp3": "SSP-RK3", "ssp54": "five-stage fourth-order SSP-RK"}
STAGES = {"ssp3": 3, "ssp54": 5}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps (the 64^3 Taylor-Green workload is run for 200)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64, help="cells per side of the periodic hex cube")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-lattice", default="650,36,128",
                    help="mixed_bl: lattice cubes along x, y, z (650,36,128 gives about 8M cells)")
    ap.add_argument("--workload", choices=("tgv_hex_p2", "tgv_tet_p3", "tgv_hex_p4", "mixed_bl"),
                    default="tgv_hex_p2",
                    help="tgv_hex_p2: the headline (FP64 plain vs FP32 + gate); tgv_tet_p3: the 48^3 x 6 "
                         "jittered-tet P3 Euler case, FP64 and FP32 throughput; tgv_hex_p4: the 64^3 hex TGV "
                         "with P4 CWENOZ5 (the paper's profiled scheme), Euler, FP64 and FP32 throughput; "
                         "mixed_bl: the 8M-cell mixed-element boundary-layer box, FP64 plain and FP32 + gate "
                         "throughput and memory")
    ap.add_argument("--gradients", choices=("green_gauss", "least_squares"), default="green_gauss",
                    help="viscous cell gradients of the Navier-Stokes workloads")
    ap.add_argument("--runs", type=int, default=1,
                    help="tgv_hex_p2: timed runs per variant, each from the initial state (value: their mean)")
    ap.add_argument("--stencil-factor", type=float, default=2.0,
                    help="tgv_tet_p3: central stencil size over K(r,3) (2: the workload's; 3: the size that is "
                         "stable at P3 on jittered tetrahedra)")
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=False,
                    help="tgv_hex_p2: time the step as one captured HIP graph replayed (the other mode is "
                         "reported beside it)")
    ap.add_argument("--integrator", choices=("ssp3", "ssp54"), default="ssp3",
                    help="tgv_hex_p2: SSP-RK3 (3 stages) or the five-stage fourth-order SSP-RK")
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-baseline-child":
        return _cpu_baseline_child(sys.argv[2], int(sys.argv[3]))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("tgv_tet_p3", "tgv_hex_p4"):
        return main_tet_p3(args) if args.workload == "tgv_tet_p3" else main_hex_p4(args)
    if args.workload == "mixed_bl":
        return main_mixed_bl(args, tuple(int(a) for a in args.mixed_lattice.split(",")))

    import torch

    from paper_2609_07387_amd import inputs, ucns

    torch.cuda.set_device(0)
    m = inputs.periodic_hex_mesh(args.n)
    U0 = inputs.tgv_initial(m)
    ph = ucns.phys(flux="hllc", viscous=True, mach=0.1, reynolds=1600.0, gradients=args.gradients)
    t0 = time.perf_counter()
    lm = ucns.Mesh(m, order=2)
    print(f"[bench] mesh build {time.perf_counter() - t0:.1f} s, {lm.n_cell} cells, {lm.n_face} faces", file=sys.stderr,
          flush=True)
    nc = lm.n_cell
    import numpy as np

    from paper_2609_07387_amd import gate

    runs = [("fp64_plain", ucns.F64, None), ("fp32", ucns.F32, None)]
    mlp = None
    if os.path.exists(gate.WEIGHTS):
        mlp = torch.tensor(np.load(gate.WEIGHTS).astype(np.float32), device="cuda")
        runs.append(("fp32_gate", ucns.F32, mlp))
    variants = {}
    for name, prec, net in runs:
        solver = ucns.Solver(lm, ph, prec, cfl=0.5, mlp=net, integrator=args.integrator)
        # each run restarts from the initial state: warm-up, then the timed steps
        per_run = []
        for _ in range(args.runs):
            U = torch.tensor(U0, dtype=torch.float64, device="cuda")
            per_run.append(time_steps(solver, U, args.steps, args.warmup, torch, graph=args.graph))
        solver.check()   # the final state is finite with positive density and pressure (host round trip)
        # the other launch mode, same window (eager launches vs one captured step replayed)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        other_solver = ucns.Solver(lm, ph, prec, cfl=0.5, mlp=net, integrator=args.integrator)
        other_ms, _ = time_steps(other_solver, U, args.steps, args.warmup, torch,
                                 graph=not args.graph and args.integrator == "ssp3")
        del other_solver
        ms = sum(r[0] for r in per_run) / len(per_run)
        wall = sum(r[1] for r in per_run) / len(per_run)
        rate = nc * STAGES[args.integrator] * args.steps / (ms / 1e3)
        # the configuration's own 200-step window (after the same warm-up),
        # reported beside the timed window when that one is shorter
        long_rate = None
        if args.steps < 200:
            U = torch.tensor(U0, dtype=torch.float64, device="cuda")
            lms, _ = time_steps(solver, U, 200, args.warmup, torch)
            solver.check()
            long_rate = nc * STAGES[args.integrator] * 200 / (lms / 1e3)
        # last, so that a profiler's last steps x stages dispatches of the
        # reconstruction kernels are this replay's timed calls
        rms, frac = time_recon_replay(solver, U0, args.steps, args.warmup, torch)
        gate = net is not None
        fused = solver.fused
        grad_mode = (2 if args.gradients == "least_squares" else 1) if fused else 0
        rbc = ((1 - frac) * recon_bytes_per_cell(lm, prec, gate=gate, grad=fused)
               + frac * recon_bytes_per_cell(lm, prec, linear=True, gate=gate, grad=fused))
        variants[name] = {"value": rate, "ms_per_step": ms / args.steps, "wall_s": wall,
                          ("ms_per_step_eager" if args.graph else "ms_per_step_graph"): other_ms / args.steps,
                          "ms_per_step_runs": [r[0] / args.steps for r in per_run],
                          "recon_ms": rms, "recon_bytes_per_cell": rbc, "recon_GBs": rbc * nc / (rms / 1e3) / 1e9,
                          "fused_gradients": fused, "grad_mode": grad_mode,
                          "step_bytes_per_cell_stage": step_bytes_per_cell(lm, prec, recon=rbc, fused=fused),
                          "path_GBs": step_bytes_per_cell(lm, prec, recon=rbc, fused=fused) * rate / 1e9}
        if net is not None:
            variants[name]["fraction_gated"] = frac
        if long_rate is not None:
            variants[name]["value_200_steps"] = long_rate
        print(f"[bench] {name}: {rate:.3e} cell-stage/s, {ms / args.steps:.3f} ms/step, recon {rms:.3f} ms"
              + (f", gated {frac:.1%}" if net is not None else "")
              + (f"; 200-step window {long_rate:.3e}" if long_rate else ""), file=sys.stderr, flush=True)
        del solver
    copy_calibration(torch)
    head = "fp32_gate" if "fp32_gate" in variants else "fp64_plain"
    hv = variants[head]
    kname = recon_kernels(head, hv["grad_mode"])
    achieved = hv["recon_GBs"]
    from paper_2609_07387_amd import prof

    rec = prof.load_traffic(os.path.join(ROOT, "profiles", TRAFFIC[head]))
    traffic = rec["bytes_per_launch"] if rec and all(k in rec["kernel"] for k in kname.split("|")) else None
    out = {
        "metric": METRIC, "value": hv["value"], "unit": "cell-stage updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if head != "fp64_plain" else "f64", "data": "synthetic",
        "config": {"workload": f"TGV {args.n}^3 periodic hex, P2 CWENOZ, HLLC, Navier-Stokes Re 1600 Mach 0.1, "
                               f"{GRAD_NAME[args.gradients]} gradients, {RK_NAME[args.integrator]} CFL 0.5, "
                               "per-step KE",
                   "cells": nc, "faces": lm.n_face,
                   "variant": head + (" (FP32 reconstruction/flux, FP64 state/RK/reductions, BF16 gate network)"
                                      if head == "fp32_gate" else "")},
        "variants": variants,
        "fp64_plain_value": variants["fp64_plain"]["value"],
        "speedup_vs_fp64_plain": hv["value"] / variants["fp64_plain"]["value"],
        "speedup_vs_fp64_plain_200_steps": (hv["value_200_steps"] / variants["fp64_plain"]["value_200_steps"]
                                            if "value_200_steps" in hv else None),
        "roofline": {"kernel": ("ucns_reconstruct_gradients" if hv["fused_gradients"] else "ucns_reconstruct")
                               + " call: " + " + ".join(kname.split("|")), "bound": "hbm",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": hv["recon_bytes_per_cell"] * nc,
                     "bytes_per_cell": hv["recon_bytes_per_cell"], "launch_ms": hv["recon_ms"],
                     "launches_timed": args.steps * STAGES[args.integrator],
                     "measured_GBs": traffic / (hv["recon_ms"] / 1e3) / 1e9 if traffic else None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def main_tet_p3(args, n=48):
    """P3 on the tetrahedral TGV (n^3 lattice cubes, 6 jittered tets each,
    1 % velocity noise), HLLC, Euler: FP64 and FP32 cell-stage updates/s and
    the reconstruction call against its byte model.  No gate (the network is
    trained at P2) and no CPU baseline (the oracle takes minutes per step
    here)."""
    import torch

    from paper_2609_07387_amd import inputs, ucns

    torch.cuda.set_device(0)
    m = inputs.kuhn_tet_mesh((n, n, n), (2.0 * math.pi,) * 3, (True,) * 3, 0.15, seed=0)
    U0 = inputs.tgv_initial(m, noise_seed=1000)
    ph = ucns.phys(flux="hllc", viscous=False)
    t0 = time.perf_counter()
    lm = ucns.Mesh(m, order=3, stencil_factor=args.stencil_factor)
    print(f"[bench] mesh build {time.perf_counter() - t0:.1f} s, {lm.n_cell} cells, {lm.n_face} faces", file=sys.stderr,
          flush=True)
    nc = lm.n_cell
    variants = {}
    for name, prec in (("fp64", ucns.F64), ("fp32", ucns.F32)):
        solver = ucns.Solver(lm, ph, prec, cfl=0.5)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        ms, wall = time_steps(solver, U, args.steps, args.warmup, torch)
        solver.check()
        rate = nc * 3 * args.steps / (ms / 1e3)
        rms, _ = time_recon_replay(solver, U0, args.steps, args.warmup, torch)
        rbc = recon_bytes_per_cell(lm, prec)
        variants[name] = {"value": rate, "ms_per_step": ms / args.steps, "wall_s": wall, "recon_ms": rms,
                          "recon_bytes_per_cell": rbc, "recon_GBs": rbc * nc / (rms / 1e3) / 1e9,
                          "step_bytes_per_cell_stage": step_bytes_per_cell(lm, prec, viscous=False),
                          "path_GBs": step_bytes_per_cell(lm, prec, viscous=False) * rate / 1e9}
        print(f"[bench] {name}: {rate:.3e} cell-stage/s, {ms / args.steps:.3f} ms/step, recon {rms:.3f} ms",
              file=sys.stderr, flush=True)
        del solver
    hv = variants["fp32"]
    out = {
        "metric": "cell-stage updates/s, P3 CWENOZ + HLLC on tets", "value": hv["value"],
        "unit": "cell-stage updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"TGV {n}^3 x 6 jittered periodic tets (+1 % velocity noise), P3 CWENOZ, HLLC, "
                               "Euler, SSP-RK3 CFL 0.5, per-step KE", "cells": nc, "faces": lm.n_face,
                   "central_stencil": f"{args.stencil_factor:g} K(r,3) cells ({lm.mc_pad} padded)",
                   "variant": "fp32 (FP32 reconstruction/flux, FP64 state/RK/reductions)"},
        "variants": variants,
        "fp64_value": variants["fp64"]["value"],
        "speedup_vs_fp64": hv["value"] / variants["fp64"]["value"],
        "roofline": {"kernel": "ucns_reconstruct call (FP32, K = 19)", "bound": "hbm", "achieved": hv["recon_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hv["recon_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": hv["recon_bytes_per_cell"] * nc,
                     "bytes_per_cell": hv["recon_bytes_per_cell"]},
    }
    print(json.dumps(out), flush=True)


def main_hex_p4(args, n=64):
    """P4 CWENOZ5 (34-term central polynomial, six quadratic sector
    polynomials, 4 x 4 face points) on the n^3 periodic hex TGV, HLLC, Euler:
    FP64 and FP32 cell-stage updates/s and the reconstruction call against
    its byte model.  The paper profiles this scheme on its TGV (Sec. 5.2).
    No gate (the network is trained at P2) and no CPU baseline (the oracle's
    P4 operator build alone takes minutes at this size)."""
    import torch

    from paper_2609_07387_amd import inputs, ucns

    torch.cuda.set_device(0)
    m = inputs.periodic_hex_mesh(n)
    U0 = inputs.tgv_initial(m)
    ph = ucns.phys(flux="hllc", viscous=False)
    t0 = time.perf_counter()
    lm = ucns.Mesh(m, order=4)
    print(f"[bench] mesh build {time.perf_counter() - t0:.1f} s, {lm.n_cell} cells, {lm.n_face} faces", file=sys.stderr,
          flush=True)
    nc = lm.n_cell
    variants = {}
    for name, prec in (("fp64", ucns.F64), ("fp32", ucns.F32)):
        solver = ucns.Solver(lm, ph, prec, cfl=0.5)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        ms, wall = time_steps(solver, U, args.steps, args.warmup, torch)
        solver.check()
        rate = nc * 3 * args.steps / (ms / 1e3)
        rms, _ = time_recon_replay(solver, U0, args.steps, args.warmup, torch)
        rbc = recon_bytes_per_cell(lm, prec)
        variants[name] = {"value": rate, "ms_per_step": ms / args.steps, "wall_s": wall, "recon_ms": rms,
                          "recon_bytes_per_cell": rbc, "recon_GBs": rbc * nc / (rms / 1e3) / 1e9,
                          "arena_GB": lm.arena_bytes(prec) / 1e9,
                          "step_bytes_per_cell_stage": step_bytes_per_cell(lm, prec, viscous=False),
                          "path_GBs": step_bytes_per_cell(lm, prec, viscous=False) * rate / 1e9}
        print(f"[bench] {name}: {rate:.3e} cell-stage/s, {ms / args.steps:.3f} ms/step, recon {rms:.3f} ms "
              f"({variants[name]['recon_GBs']:.0f} GB/s algorithmic)", file=sys.stderr, flush=True)
        del solver
        lm.release()
        torch.cuda.empty_cache()
    hv = variants["fp32"]
    out = {
        "metric": "cell-stage updates/s, P4 CWENOZ5 + HLLC on hexahedra", "value": hv["value"],
        "unit": "cell-stage updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"TGV {n}^3 periodic hex, P4 CWENOZ5 (34-term central, 6 quadratic sector "
                               "polynomials, 4 x 4 face points), HLLC, Euler, SSP-RK3 CFL 0.5, per-step KE",
                   "cells": nc, "faces": lm.n_face, "central_stencil": lm.mc_pad, "sector_stencil": lm.md_pad,
                   "variant": "fp32 (FP32 reconstruction/flux, FP64 state/RK/reductions)"},
        "variants": variants,
        "fp64_value": variants["fp64"]["value"],
        "speedup_vs_fp64": hv["value"] / variants["fp64"]["value"],
        "roofline": {"kernel": "ucns_reconstruct call (P4, FP32)", "bound": "hbm", "achieved": hv["recon_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hv["recon_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": hv["recon_bytes_per_cell"] * nc,
                     "bytes_per_cell": hv["recon_bytes_per_cell"]},
    }
    print(json.dumps(out), flush=True)


def main_mixed_bl(args, n=(650, 36, 128)):
    """The mixed-element boundary-layer box (about 8M cells: 60 % tetrahedra,
    25 % prisms, 15 % hexahedra, pyramids at the hexahedron-tetrahedron
    interfaces), P2 CWENOZ, HLLC, Navier-Stokes at Mach 0.8 and Re 1e6 per
    unit length, impulsive start from the free stream over a no-slip bumped
    wall: FP64 plain and FP32 + gate cell-stage updates/s and the memory each
    takes (no CPU baseline: the oracle takes minutes per step here)."""
    import resource

    import numpy as np
    import torch

    from paper_2609_07387_amd import gate, inputs, ucns

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    m = inputs.mixed_bl_mesh(n, lengths=(4.0, 0.3, 0.5), hex_cols=(n[0] // 5, n[0] // 5))
    mix = {name: int((m.ctype == t).sum()) for name, t in (("tet", inputs.TET), ("prism", inputs.PRISM),
                                                           ("hex", inputs.HEX), ("pyramid", inputs.PYR))}
    U0 = inputs.bl_initial(m, mach=0.8, amp=0.0)
    ph = ucns.phys(flux="hllc", viscous=True, mach=0.8, reynolds=1e6, gradients=args.gradients)
    free = U0[:, 0]
    bcs = ucns.bc({1: (ucns.BC_DIRICHLET, free), 2: (ucns.BC_TRANSMISSIVE, None), 3: (ucns.BC_WALL, None),
                   4: (ucns.BC_DIRICHLET, free)})
    t1 = time.perf_counter()
    print(f"[bench] {m.n_cell} cells generated in {t1 - t0:.1f} s; building operators", file=sys.stderr, flush=True)
    lm = ucns.Mesh(m, order=2)
    print(f"[bench] mesh generated in {t1 - t0:.1f} s, built in {time.perf_counter() - t1:.1f} s: {lm.n_cell} cells "
          f"{mix}, {lm.n_face} faces", file=sys.stderr, flush=True)
    nc = lm.n_cell
    mlp = torch.tensor(np.load(gate.WEIGHTS).astype(np.float32), device="cuda")
    variants = {}
    for name, prec, net in (("fp64_plain", ucns.F64, None), ("fp32_gate", ucns.F32, mlp)):
        torch.cuda.reset_peak_memory_stats()
        solver = ucns.Solver(lm, ph, prec, bcs, cfl=0.5, mlp=net)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        ms, wall = time_steps(solver, U, args.steps, args.warmup, torch)
        solver.check()   # finite, positive density and pressure (UCNS_ENUM otherwise)
        rate = nc * 3 * args.steps / (ms / 1e3)
        frac = float(solver.ws.mask_out.float().mean()) if net is not None else 0.0
        variants[name] = {"value": rate, "ms_per_step": ms / args.steps, "wall_s": wall,
                          "arena_GB": lm.arena_bytes(prec) / 1e9,
                          "device_peak_GB": torch.cuda.max_memory_allocated() / 1e9,
                          "finite": bool(torch.isfinite(U).all())}
        if net is not None:
            variants[name]["fraction_gated"] = frac
        print(f"[bench] {name}: {rate:.3e} cell-stage/s, {ms / args.steps:.3f} ms/step"
              + (f", gated {frac:.1%}" if net is not None else ""), file=sys.stderr, flush=True)
        del solver, U
    hv = variants["fp32_gate"]
    out = {
        "metric": "cell-stage updates/s, P2 CWENOZ + HLLC + viscous on a mixed-element mesh",
        "value": hv["value"], "unit": "cell-stage updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"mixed-element boundary-layer box {n[0]}x{n[1]}x{n[2]} lattice: hexahedral "
                               "inflow/outflow blocks, 20 prism layers (growth 1.2) on a bumped no-slip wall, "
                               "tetrahedra above, pyramids at the interfaces; P2 CWENOZ, HLLC, Navier-Stokes "
                               f"Mach 0.8, Re 1e6, {GRAD_NAME[args.gradients]} gradients, SSP-RK3 CFL 0.5, "
                               "per-step KE", "cells": nc, "faces": lm.n_face,
                   "cell_mix": mix, "variant": "fp32_gate"},
        "variants": variants,
        "fp64_plain_value": variants["fp64_plain"]["value"],
        "speedup_vs_fp64_plain": hv["value"] / variants["fp64_plain"]["value"],
        "memory": {"host_peak_GB": resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6,
                   "device_GB_fp64": variants["fp64_plain"]["device_peak_GB"],
                   "device_GB_fp32_gate": hv["device_peak_GB"], "device_capacity_GB": 288},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
