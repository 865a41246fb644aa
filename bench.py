"""Benchmark of the explicit residual evaluation on one MI355X.

Workload: periodic 64^3 hexahedral Taylor-Green vortex (262,144 cells) at
Mach 0.1, Navier-Stokes Re 1600, P2 CWENOZ reconstruction, HLLC, Green-Gauss
viscous gradients, SSP-RK3 at CFL 0.5, with the per-step kinetic-energy
reduction.  A step = dt + 3 x (reconstruct, gradients, face flux, residual +
RK stage) + KE, all through the C ABI on one stream; inputs already resident
in HBM when the timed region starts.

Prints one JSON line: the headline variant's cell-stage updates/s, both
variants (FP64 plain and FP32 reconstruction/flux), the roofline of the
dominant kernel (reconstruction) timed with HIP events on its own stream, and
the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-stage updates/s, P2 CWENO+HLLC: FP64 plain vs FP32+MLP gate; % HBM peak"


def recon_bytes_per_cell(lm, precision, gated=False):
    """Algorithmic HBM bytes of one reconstruction of one cell: every operator
    value and index read once, the cell's own state read once, its face-point
    states written once (neighbour states are re-reads of resident data)."""
    t = 8 if precision == 0 else 4
    K, MC, MD, ND, NF, Q = lm.K, lm.mc_pad, max(1, lm.md_pad), max(1, lm.nd_max), lm.nfmax, lm.qmax
    ops = K * MC + K * (K + 1) // 2 + NF * Q * K + (0 if gated else ND * 3 * MD)
    idx = MC + NF + (0 if gated else ND * MD)
    return t * ops + 4 * idx + 1 + 40 + t * 5 * NF * Q + NF


def step_bytes_per_cell(lm, precision, viscous=True):
    """Algorithmic HBM bytes of one stage of the whole path per cell."""
    t = 8 if precision == 0 else 4
    faces_per_cell = lm.n_face / lm.n_cell
    Q, NF = lm.qmax, lm.nfmax
    recon = recon_bytes_per_cell(lm, precision)
    flux = faces_per_cell * (2 * Q * 5 * t + t * (7 + Q) + 9 + 5 * t + (24 * t if viscous else 0))
    grad = (40 + 4 * NF + 12 * t + faces_per_cell * (8 + 4 * t)) if viscous else 0
    resid = 4 * NF + 5 * t * NF + 8 + 40 * 3
    return recon + flux + grad + resid


def time_steps(solver, U, steps, warmup, torch):
    for _ in range(warmup):
        solver.step(U, ke=True)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        solver.step(U, ke=True)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall


def time_recon(lm, ph, U, precision, fs, flags, reps, torch, ucns):
    s = torch.cuda.current_stream()
    for _ in range(3):
        ucns.reconstruct(lm, ph, U, precision, fs, None, flags)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ucns.reconstruct(lm, ph, U, precision, fs, None, flags)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(seconds=12.0):
    """The FP64 oracle as it stands, on this host: 32^3 hex TGV with the same
    scheme (per-cell work is that of the 64^3 workload), SSP-RK3 steps until
    `seconds` have elapsed; mesh build excluded."""
    import oracle
    from paper_2609_07387_amd import inputs

    m = inputs.periodic_hex_mesh(32)
    U = inputs.tgv_initial(m)
    om = oracle.OracleMesh(m, order=2)
    ph = oracle.phys(flux="hllc", viscous=True)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and steps < 400:
        U, _, _ = om.run(U, ph, 0.5, 1)
        steps += 1
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": m.n_cell * 3 * steps / dt, "unit": "cell-stage updates/s", "cores": cores, "kind": "oracle",
            "sample": f"32^3 periodic hex TGV, same scheme (P2 CWENOZ, HLLC, NS, Green-Gauss), {steps} SSP-RK3 "
                      f"steps in {dt:.1f} s, mesh build excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="cells per side of the periodic hex cube")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_07387_amd import inputs, ucns

    torch.cuda.set_device(0)
    m = inputs.periodic_hex_mesh(args.n)
    U0 = inputs.tgv_initial(m)
    ph = ucns.phys(flux="hllc", viscous=True, mach=0.1, reynolds=1600.0)
    t0 = time.perf_counter()
    lm = ucns.Mesh(m, order=2)
    print(f"[bench] mesh build {time.perf_counter() - t0:.1f} s, {lm.n_cell} cells, {lm.n_face} faces", file=sys.stderr,
          flush=True)
    nc = lm.n_cell
    variants = {}
    for name, prec in (("fp64_plain", ucns.F64), ("fp32", ucns.F32)):
        solver = ucns.Solver(lm, ph, prec, cfl=0.5)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        ms, wall = time_steps(solver, U, args.steps, args.warmup, torch)
        rate = nc * 3 * args.steps / (ms / 1e3)
        rms = time_recon(lm, ph, U, prec, solver.ws.face_state, solver.ws.flags, 20, torch, ucns)
        rb = recon_bytes_per_cell(lm, prec) * nc
        variants[name] = {"value": rate, "ms_per_step": ms / args.steps, "wall_s": wall,
                          "recon_ms": rms, "recon_GBs": rb / (rms / 1e3) / 1e9,
                          "step_bytes_per_cell_stage": step_bytes_per_cell(lm, prec),
                          "path_GBs": step_bytes_per_cell(lm, prec) * rate / 1e9}
        print(f"[bench] {name}: {rate:.3e} cell-stage/s, {ms / args.steps:.3f} ms/step, recon {rms:.3f} ms",
              file=sys.stderr, flush=True)
        del solver
    head = "fp64_plain"
    hv = variants[head]
    recon_prec = ucns.F64
    achieved = recon_bytes_per_cell(lm, recon_prec) * nc / (hv["recon_ms"] / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": hv["value"], "unit": "cell-stage updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"TGV {args.n}^3 periodic hex, P2 CWENOZ, HLLC, Navier-Stokes Re 1600 Mach 0.1, "
                               "Green-Gauss, SSP-RK3 CFL 0.5, per-step KE", "cells": nc, "faces": lm.n_face,
                   "variant": head},
        "variants": variants,
        "speedup_fp32_over_fp64": variants["fp32"]["value"] / variants["fp64_plain"]["value"],
        "roofline": {"kernel": "reconstruct_kernel<double,9>", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_cell": recon_bytes_per_cell(lm, recon_prec)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
