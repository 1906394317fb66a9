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

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (an FMA counts 2)
STEP_ALGO_BYTES = 320.0         # bytes per zone-cycle a fully fused VL2 FP64 step must move

# Algorithmic work per cell of one launch of each kernel class.  Bytes: every array the
# kernel needs read once, every array it produces written once (FP64).  Flops: the
# FP64 add/sub/mul/div/sqrt of the method's formulas counted once per cell (PPM shared
# between the two faces a cell touches; compares, min/max and selects not counted).
KERNEL_ALGO = {
    # state (8 fields) in; 3 x 7 face fields + 3 cell E fields out
    "mhd_flux_corrector": {"bytes": (8 + 24) * 8, "flops": 1701},  # PPM + HLLD, 3 faces
    "mhd_flux_predictor": {"bytes": (8 + 24) * 8, "flops": 1155},  # donor cell + HLLD
    # 24 face/cell fields + base register (8) in; 8 fields out
    "mhd_ct_update_corrector": {"bytes": (24 + 8 + 8) * 8, "flops": 192},
    "mhd_ct_update_predictor": {"bytes": (24 + 8 + 8) * 8, "flops": 120},
    "cfl": {"bytes": 8 * 8, "flops": 72},
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


def fp32_leg(n, state, warm_dts, dts, ref64):
    """The FP32-bulk form (FP64 total energy) on the same workload and the same dt
    sequence as the FP64 run (each step still reads its own CFL step, as in the FP64
    loop); reports its throughput and the relative L1 difference of each conserved
    class to the FP64 state after the same steps."""
    import torch

    from paper_2608_14048_amd import Sim

    print("[bench] FP32-bulk leg", file=sys.stderr, flush=True)
    sim = Sim((n, n, n), scheme=dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3,
                                     prec="fp32_bulk"))
    sim.set_state(state)
    for dt in warm_dts:
        sim.dt_cfl()
        sim.step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in dts:
        sim.dt_cfl()
        sim.step(dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    got = sim.state(device=True).reshape(8, -1)
    ref = ref64.reshape(8, -1)
    rows = {"rho": [0], "M": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    l1 = {k: float((got[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for k, v in rows.items()}
    sim.close()
    steps = len(dts)
    return {"value": round(n ** 3 * steps / el / 1e6, 2), "unit": "Mzone-cycles/s",
            "ms_per_step": round(el * 1e3 / steps, 4), "dtype": "f32 (E in f64)",
            "l1_rel_vs_fp64": {k: float(f"{v:.3e}") for k, v in l1.items()},
            "compared_after_steps": len(warm_dts) + steps}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 2 GiB device copy three times (the calibration "
                         "launch for HBM byte counters)")
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

    if args.copy_probe:
        # 2 GiB read + 2 GiB written per launch
        src = torch.ones(1 << 28, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n = args.n
    print(f"[bench] building the {n}^3 initial state", file=sys.stderr, flush=True)
    state = I.turbulence(n, seed=args.seed)

    sim = Sim((n, n, n), scheme=dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3))
    sim.set_state(state)
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    warm_dts = []
    for _ in range(args.warmup):
        dt = sim.dt_cfl()
        sim.step(dt)
        warm_dts.append(dt)
    torch.cuda.synchronize()
    # events around every launch of the timed region (16 launches per step at most)
    sim.timing(capacity=32 * args.steps + 64)
    sim.timing_read()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    dts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dt = sim.dt_cfl()
        sim.step(dt)
        dts.append(dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = sim.timing_read()
    sim.timing(0)
    elapsed = t1 - t0
    ncell = n ** 3
    value = ncell * args.steps / elapsed / 1e6
    ms_per_step = elapsed * 1e3 / args.steps

    # roofline of the kernel class with the largest device time, against the resource
    # it is closer to saturating (HBM bytes or FP64 vector flops)
    dominant = max(times, key=lambda k: times[k][0])
    total_ms, launches = times[dominant]
    avg_s = total_ms / launches * 1e-3
    work = KERNEL_ALGO.get(dominant, {"bytes": 0, "flops": 0})
    gbs = work["bytes"] * ncell / avg_s / 1e9
    tfl = work["flops"] * ncell / avg_s / 1e12
    f_hbm, f_alu = gbs / HBM_PEAK_GBS, tfl / FP64_VECTOR_PEAK_TFLOPS
    traffic = measured_traffic(dominant, ncell)
    if f_alu > f_hbm:
        roofline = {"bound": "alu", "achieved": round(tfl, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(f_alu, 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(f_hbm, 4)}
    roofline.update({"traffic": traffic, "kernel": dominant,
                     "avg_launch_ms": round(total_ms / launches, 4), "launches": launches,
                     "hbm_frac": round(f_hbm, 4), "alu_frac": round(f_alu, 4)})
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
    if not args.no_fp32:
        out["fp32_bulk"] = fp32_leg(n, state, warm_dts, dts, sim.state(device=True))
    sim.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, state, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
