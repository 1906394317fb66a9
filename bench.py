#!/usr/bin/env python3
"""Throughput of the 3D CT-MHD Godunov step on one MI355X.

Workload: decaying MHD turbulence on a periodic 256^3 box (seed 0; lognormal density,
k^-2 velocity field at rms Mach 1, random-potential field at plasma beta 1), the
VL2 integrator with PPM reconstruction, the HLLD Riemann solver and constrained
transport, Courant 0.3, FP64.  One step = {dt = CFL step of the state (8-byte read);
advance by dt}; every step does the whole update on the GPU with the state resident in
HBM.  The metric counts each cell once per cycle (Mzone-cycles/s).

Prints one JSON line.  Besides the throughput it reports the roofline of the kernel
class that takes most device time (HIP events on the library's stream over the timed
region) and the CPU oracle timed on this host on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
STEP_ALGO_BYTES = 320.0        # bytes per zone-cycle a fused VL2 FP64 step must move

# Algorithmic HBM bytes per cell of one launch of each kernel class: every array the
# kernel needs read once, every array it produces written once (FP64).
KERNEL_ALGO_BYTES = {
    "mhd_prims": (8 + 8) * 8,              # conserved + face fields in, 8 primitives out
    "mhd_flux_predictor": (7 + 1 + 7) * 8,  # 7 face-frame primitives + normal B in, 7 out
    "mhd_flux_corrector": (7 + 1 + 7) * 8,
    "mhd_edges": (6 + 9 + 3) * 8,          # v, B_cc; mass flux + 2 face E per sweep; 3 edge E
    "mhd_update": (8 + 8 + 15 + 3 + 8) * 8,  # in, base, 5 fluxes x 3 sweeps, 3 edge E; out
    "cfl": 8 * 8,
}

WORKLOAD = "decaying MHD turbulence, periodic {n}^3, VL2+PPM+HLLD+CT, CFL 0.3, seed 0"


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_14048_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, n_cells: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel class, if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        ent = rec.get("kernels", {}).get(kernel)
        if not ent or rec.get("source_digest") != source_digest() or rec.get("n_cells") != n_cells:
            return None
        return float(ent["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(n: int, state, max_seconds: float = 30.0):
    """The oracle as it stands on a bounded sample: as many steps of the same workload
    as fit in about max_seconds (at least one)."""
    import oracle

    cfg = oracle.make_cfg((n, n, n), recon="ppm", riemann="hlld", integ="vl2", courant=0.3)
    s = state.copy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        dt = oracle.dt_cfl(cfg, s)
        s = oracle.step(cfg, s, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el * (steps + 1) / steps > max_seconds:
            break
    value = n ** 3 * steps / el / 1e6
    return {"value": round(value, 4), "unit": "Mzone-cycles/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} step(s) of the {n}^3 workload from the same initial state "
                      f"({el:.1f} s, OpenMP over k-planes)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2608_14048_amd import Sim
    from paper_2608_14048_amd import inputs as I

    n = args.n
    print(f"[bench] building the {n}^3 initial state", file=sys.stderr, flush=True)
    state = I.turbulence(n, seed=args.seed)

    sim = Sim((n, n, n), scheme=dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3))
    sim.set_state(state)
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sim.step(sim.dt_cfl())
    torch.cuda.synchronize()
    # events around every launch of the timed region (16 launches per step at most)
    sim.timing(capacity=32 * args.steps + 64)
    sim.timing_read()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.step(sim.dt_cfl())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = sim.timing_read()
    sim.timing(0)
    elapsed = t1 - t0
    ncell = n ** 3
    value = ncell * args.steps / elapsed / 1e6
    ms_per_step = elapsed * 1e3 / args.steps

    # roofline of the kernel class with the largest device time
    dominant = max(times, key=lambda k: times[k][0])
    total_ms, launches = times[dominant]
    avg_s = total_ms / launches * 1e-3
    algo = KERNEL_ALGO_BYTES.get(dominant, 0) * ncell
    achieved = algo / avg_s / 1e9
    traffic = measured_traffic(dominant, ncell)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_ms": round(total_ms / launches, 4),
                "launches": launches}
    kernel_ms = {k: round(v[0] / args.steps, 4) for k, v in sorted(times.items())}

    out = {
        "metric": "Mzone-cycles/s, 3D CT-MHD VL2+HLLD 256^3, FP64 vs FP32; % HBM roofline",
        "value": round(value, 2),
        "unit": "Mzone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD.format(n=n), "grid": [n, n, n], "integrator": "vl2",
                   "reconstruction": "ppm", "riemann": "hlld", "precision": "fp64",
                   "courant": 0.3, "parallelism": "single GPU"},
        "roofline": roofline,
        "step_hbm_roofline": {"algo_bytes_per_zone_cycle": STEP_ALGO_BYTES,
                              "frac": round(value * 1e6 * STEP_ALGO_BYTES / (HBM_PEAK_GBS * 1e9), 4)},
        "kernel_ms_per_step": kernel_ms,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, state, args.cpu_seconds)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
