"""Benchmark of the MAFOD hot path on one MI355X.

A step is one mf4d_filter call over the roofline-scale workload: a 4096 x 4096
float32 image with 64 bright and dark creases (widths 1-16 px, noise
N(0, 0.05)), 8 log-spaced scales 1..16, ridge+valley mode, 30 FED cycles of
20 substeps -- scale selection, normalised Hessian and every substep included,
with the input already resident in HBM.

Prints one JSON line:
  value     Mpixel-FED-substeps/s of the whole filter (H W M n per step / time)
  roofline  the fused FED substep kernel: algorithmic bytes per launch
            (20 B/px: u read 4, H_rho read 12, u write 4) / its average launch
            time, timed with HIP events on the stream it is launched on
  cpu_baseline  the FP64 oracle on a bounded sample (one cycle of the same image)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
SUBSTEP_BYTES_PER_PX = 20  # u in 4 + H_rho in 12 + u out 4


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_stream(torch, fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    s, e = _events(torch)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="creases4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1611_06906_amd import mf4d, synth

    w = synth.WORKLOADS[args.workload]()
    t0 = time.time()
    u_np = w.image()
    print(f"[bench] workload {w.name} {w.H}x{w.W} generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    p = mf4d.Params.from_workload(w)
    u_in = torch.from_numpy(u_np).to(dev)
    u_out = torch.empty_like(u_in)
    ws = mf4d.workspace(w.H, w.W, p, dev)
    torch.cuda.synchronize()

    step = lambda: mf4d.mf4d_filter(u_in, u_out, p, ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K whole-filter steps (single rank: no barrier needed)
    ms = time_stream(torch, step, args.steps)
    px_sub = w.H * w.W * w.cycles * w.substeps
    value = px_sub / (ms * 1e-3) / 1e6
    print(f"[bench] {args.steps} steps, {ms:.2f} ms/step, {value:.0f} Mpx-substeps/s", file=sys.stderr,
          flush=True)

    # roofline of the fused FED substep: same kernel and shapes, H_rho of the workload
    n, taus = mf4d.mf4d_fed_plan(p)
    hrho = torch.empty((3, w.H, w.W), dtype=torch.float32, device=dev)
    idx = torch.empty((w.H, w.W), dtype=torch.uint8, device=dev)
    mf4d.mf4d_scale_select(u_in, p, idx, None, None, ws)
    mf4d.mf4d_tensor(u_in, idx, p, hrho, None, ws)
    uc = u_in.clone()
    ut = torch.empty_like(uc)
    cyc = lambda: mf4d.mf4d_fed_cycle(uc, ut, hrho, p, taus)
    cyc()
    reps = 5
    ms_cycle = time_stream(torch, cyc, reps)
    ms_substep = ms_cycle / n   # n even: no copy-back launch in the cycle
    achieved = SUBSTEP_BYTES_PER_PX * w.H * w.W / (ms_substep * 1e-3)
    roofline = {"bound": "hbm", "kernel": "fed_substep_kernel", "achieved": achieved / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                "us_per_launch": ms_substep * 1e3, "bytes_per_px": SUBSTEP_BYTES_PER_PX}

    # one single-step cycle: a substep plus the plain copy of H*W floats back
    # into u (4 B read + 4 B write per pixel), the reference for HBM counters
    mf4d.mf4d_fed_cycle(uc, ut, hrho, p, taus[:1])
    torch.cuda.synchronize()

    stages = None
    if not args.no_stages:
        sel_ms = time_stream(torch, lambda: mf4d.mf4d_scale_select(u_in, p, idx, None, None, ws), 3)
        ten_ms = time_stream(torch, lambda: mf4d.mf4d_tensor(u_in, idx, p, hrho, None, ws), 3)
        stages = {"scale_select_ms": sel_ms, "tensor_incl_sweep_ms": ten_ms,
                  "fed_cycle_ms": ms_cycle, "cycles": w.cycles}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        omp = int(os.environ.get("OMP_NUM_THREADS", cores))
        t1 = time.time()
        oracle.filter(u_np, w.sigmas, w.mode, lam=w.lam, rho=w.rho, beta=w.beta, cycles=1,
                      substeps=w.substeps, tau_max=w.tau_max)
        dt = time.time() - t1
        cpu = {"value": w.H * w.W * w.substeps / dt / 1e6, "unit": "Mpixel-FED-substeps/s",
               "cores": min(omp, cores), "kind": "oracle",
               "sample": f"1 of {w.cycles} cycles ({w.substeps} substeps) of the full {w.H}x{w.W} image, "
                         f"FP64, {dt:.1f} s"}

    out = {
        "metric": "Mpixel-FED-substeps/s and % HBM roofline, plain vs batched/learned @ oracle tol",
        "value": value,
        "unit": "Mpixel-FED-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.H}x{w.W} creases, {len(w.sigmas)} scales 1-16, "
                               f"ridge+valley, {w.cycles} FED cycles x {w.substeps} substeps, plain path",
                   "H": w.H, "W": w.W, "cycles": w.cycles, "substeps": w.substeps,
                   "nscales": len(w.sigmas), "mode": "both", "path": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages": stages,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
