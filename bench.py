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
Side legs, each on its own workload and reported in its own object: the FP32-bulk form
of the same run, the gas + 8 dust IMEX2P step at 192^3, and the RK2+PLM+HLLE oblique
linear wave on a 512 x 512 x 256 box (the scheme and box of the paper's performance
table), and 512 uneven meshblocks as one batch against the same blocks launched one by
one, and the learned closure on held-out seeds.  The dust leg also runs its FP32 form
(FP32 state and explicit part, FP64 drag solve) on the same dt sequence.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--no-cpu-baseline]
                       [--no-fp32] [--no-dust] [--no-paper-config] [--no-batch] [--no-closure]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (an FMA counts 2)
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, packed (the kernels here issue no packed FP32)
STEP_ALGO_BYTES = 320.0         # bytes per zone-cycle a fully fused VL2 FP64 step must move
STEP_ALGO_BYTES_FP32 = 180.0    # the same for the FP32-bulk form (7 FP32 fields + FP64 E)

# Algorithmic bytes per cell of each stage of the VL2 step (the traffic model of the
# fused step: each stage reads its input register once, the corrector also the base
# register, and writes one register): predictor 8 + 8 fields, corrector 8 + 8 + 8.  The
# roofline of the dominant kernel divides its stage's bytes by that kernel's time (the
# kernel does the stage's reading and most of its writing; the CT kernel beside it
# finishes the face fields).
STAGE_ALGO_BYTES = {"predictor": 128.0, "corrector": 192.0}
STAGE_ALGO_BYTES_FP32 = {"predictor": 72.0, "corrector": 108.0}

# Algorithmic work per cell of one launch of each kernel class.  Bytes: every array the
# kernel needs read once, every array it produces written once (FP64).  Flops: the
# FP64 add/sub/mul/div/sqrt of the method's formulas counted once per cell (PPM shared
# between the two faces a cell touches; compares, min/max and selects not counted).
# stage: which stage's bytes the dominant-kernel roofline uses.
KERNEL_ALGO = {
    # stage input (8 fields) and, corrector, the base register's cell fields (5) in;
    # 5 cell fields, 9 face fields and 3 cell E fields out
    "mhd_flux_update_corrector": {"bytes": (8 + 5 + 5 + 12) * 8, "flops": 1701 + 40, "stage": "corrector"},
    "mhd_flux_update_predictor": {"bytes": (8 + 5 + 12) * 8, "flops": 1155 + 40, "stage": "predictor"},
    # 12 face/cell fields and the base face fields (3) in, 3 face fields out; the
    # corrector also reads the 5 new cell fields for the time step
    "mhd_ct_corrector": {"bytes": (12 + 3 + 3 + 5) * 8, "flops": 152, "stage": "corrector"},
    "mhd_ct_predictor": {"bytes": (12 + 3 + 3) * 8, "flops": 80, "stage": "predictor"},
    "cfl": {"bytes": 8 * 8, "flops": 72},
}

# FP32-bulk form: a state is 7 FP32 fields + FP64 E = 36 B (cell fields: 3 x 4 + 8 = 20
# B; face fields 12 B), a face or cell-E field 4 B; the flops are those of the FP64
# table, in FP32 (E's update in FP64)
KERNEL_ALGO_FP32 = {
    "mhd_flux_update_corrector": {"bytes": 36 + 20 + 20 + 12 * 4, "flops": 1741, "stage": "corrector"},
    "mhd_flux_update_predictor": {"bytes": 36 + 20 + 12 * 4, "flops": 1195, "stage": "predictor"},
    "mhd_ct_corrector": {"bytes": 12 * 4 + 12 + 12 + 20, "flops": 152, "stage": "corrector"},
    "mhd_ct_predictor": {"bytes": 12 * 4 + 12 + 12, "flops": 80, "stage": "predictor"},
    "cfl": {"bytes": 36, "flops": 72},
}

# Gas + dust IMEX2P kernels (36 fields per state at 8 dust species, 27 of them momenta),
# bytes per cell: every array the kernel needs read once, every array it produces
# written once.  The step's own minimum (stage 1 reads u and writes U1, stage 2 reads
# u and U1 and writes u) is 5 x 36 fields; the four launches move 342 fields.
DUST_FIELDS, DUST_MOM = 36, 27
DUST_STEP_ALGO_BYTES = 5 * DUST_FIELDS * 8


def dust_kernel_algo(word: int) -> dict:
    """Algorithmic bytes per cell of each dust kernel class for fields of `word` bytes."""
    return {
        "dust_fluid_pass_stage1": {"bytes": 2 * DUST_FIELDS * word, "stage": "stage1"},             # u in, X out
        "dust_fluid_pass_stage2": {"bytes": 3 * DUST_FIELDS * word, "stage": "stage2"},             # U1, u in, X out
        "dust_drag_stage1": {"bytes": (DUST_FIELDS + DUST_MOM) * word, "stage": "stage1"},          # X in, momenta out
        "dust_drag_cfl_stage2": {"bytes": (2 * DUST_FIELDS + DUST_MOM) * word, "stage": "stage2"},  # X, U1 in, momenta out
        "cfl": {"bytes": DUST_FIELDS * 8},
    }


DUST_KERNEL_ALGO = dust_kernel_algo(8)
DUST_KERNEL_ALGO_FP32 = dust_kernel_algo(4)
# the fused-step traffic model per stage: stage 1 reads u and writes U1, stage 2 reads u
# and U1 and writes u (1440 B per zone-cycle in FP64 at 8 species)
DUST_STAGE_BYTES = {"stage1": 2 * DUST_FIELDS * 8.0, "stage2": 3 * DUST_FIELDS * 8.0}
DUST_STAGE_BYTES_FP32 = {"stage1": 2 * DUST_FIELDS * 4.0, "stage2": 3 * DUST_FIELDS * 4.0}

WORKLOAD = "decaying MHD turbulence, periodic {n}^3, VL2+PPM+HLLD+CT, CFL 0.3, seed 0"


# the sources that define the kernels whose traffic profiles/traffic.json records
DIGEST_SOURCES = ("common.hpp", "launch.hpp", "physics.hpp", "mhd_tiles.hpp", "mhd_fused.hip",
                  "dust_kernels.hip", "reduce.hip", "api.hip")


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_14048_amd", "csrc")
    for name in DIGEST_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str, n_cells: int):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter summary
    (calibrated FETCH_SIZE + WRITE_SIZE), if it was taken on the current kernel sources
    and the same workload size (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_digest") != source_digest():
            return None
        wl = rec.get("workloads", {}).get(workload, {})
        ent = wl.get("kernels", {}).get(kernel)
        if not ent or wl.get("n_cells") != n_cells:
            return None
        return float(ent["bytes_per_launch"])
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def timed_run(sim, steps: int, warmup: int, dts_in=None):
    """{dt = CFL step; step(dt)} warmup times, then steps times under HIP-event timing of
    every launch.  With dts_in the given dt sequence (warm-up first) is stepped instead,
    each step still reading its own CFL step.  Returns (seconds, per-class event times,
    warm-up dts, timed dts)."""
    import torch

    warm, dts = [], []
    for k in range(warmup):
        dt = sim.dt_cfl()
        dt = dts_in[k] if dts_in is not None else dt
        sim.step(dt)
        warm.append(dt)
    torch.cuda.synchronize()
    sim.timing(capacity=32 * steps + 64)
    sim.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        dt = sim.dt_cfl()
        dt = dts_in[warmup + k] if dts_in is not None else dt
        sim.step(dt)
        dts.append(dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    times = sim.timing_read()
    sim.timing(0)
    return el, times, warm, dts


def measured_counters(workload: str, kernel: str):
    """VALU work and issue rates of a kernel class from the committed counter summary, if
    it was taken on the current kernel sources (else None): VALU and FP64-arithmetic
    wave instructions per cell, and per CU-cycle at 2.4 GHz and at the clock the kernel
    ran at (GRBM_GUI_ACTIVE over its duration); a CU issues at most one VALU wave
    instruction per cycle (four SIMDs, four cycles per wave64 instruction)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_digest") != source_digest():
            return None
        ent = rec.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel, {})
        out = {k: ent[k] for k in ("valu_per_cell", "fp64_per_cell", "valu_issue", "fp64_issue", "clock_ghz",
                                   "valu_issue_at_clock", "fp64_issue_at_clock") if k in ent}
        return out or None
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def kernel_roofline(times, table, ncell, workload, stage_bytes):
    """HBM roofline of the kernel class with the largest device time: the algorithmic
    bytes of its stage (the fused-step traffic model, bytes per cell x cells) per
    average launch duration, against the 8 TB/s peak.  Beside it: the kernel's own
    minimum bytes, its measured bytes per launch (rocprof FETCH_SIZE + WRITE_SIZE, when
    taken on the current sources) and its VALU issue rates from the SQ counters."""
    dominant = max(times, key=lambda k: times[k][0])
    total_ms, launches = times[dominant]
    avg_s = total_ms / launches * 1e-3
    work = table.get(dominant, {"bytes": 0})
    per_cell = stage_bytes.get(work.get("stage"), work["bytes"])
    gbs = per_cell * ncell / avg_s / 1e9
    traffic = measured_traffic(workload, dominant, ncell)
    rf = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dominant,
          "algo_bytes_per_cell": per_cell,
          "algo_basis": f"{work.get('stage', 'kernel')} stage of the fused-step traffic model",
          "kernel_min_bytes_per_cell": work["bytes"],
          "avg_launch_ms": round(total_ms / launches, 4), "launches": launches}
    if traffic is not None:
        rf["traffic_over_algo"] = round(traffic / (per_cell * ncell), 3)
    cnt = measured_counters(workload, dominant)
    if cnt:
        rf["counters"] = cnt
    return rf


def step_traffic(workload: str, times, ncell: int, steps: int, algo_bytes_per_cell: float):
    """Measured HBM bytes of one step (every kernel class, per-launch bytes x launches
    per step) over the step's algorithmic bytes, when the counters were taken on the
    current sources (else None)."""
    total = 0.0
    for k, (_, launches) in times.items():
        b = measured_traffic(workload, k, ncell)
        if b is None:
            return None
        total += b * launches / steps
    return {"bytes_per_step": round(total), "over_algo": round(total / (algo_bytes_per_cell * ncell), 3)}


def dust_leg(n: int, steps: int, warmup: int, seed: int = 0, fp32: bool = True):
    """Gas + 8 dust fluids, isothermal gas, IMEX2P with PLM, isothermal HLLE and
    pressureless Rusanov, gas acceleration 0.05 x^, n^3 periodic, FP64; then (fp32) the
    FP32 form (FP32 state and explicit part, FP64 drag solve) on the same dt sequence,
    with the relative L1 difference of each class to the FP64 state."""
    from paper_2608_14048_amd import Sim
    from paper_2608_14048_amd import inputs as I

    print(f"[bench] dust leg {n}^3", file=sys.stderr, flush=True)
    state, ts = I.dust_drift(n, seed=seed)
    physics = dict(eos="isothermal_hydro", cs=1.0, tstop=tuple(ts), gacc=(0.05, 0.0, 0.0))
    scheme = dict(recon="plm", riemann="hlle", integ="imex2p", courant=0.3)
    sim = Sim((n, n, n), physics=physics, scheme=scheme)
    sim.set_state(state)
    el, times, warm, dts = timed_run(sim, steps, warmup)
    ref = sim.state(device=True) if fp32 else None
    sim.close()
    ncell = n ** 3
    value = ncell * steps / el / 1e6
    out = {"workload": f"gas + 8 dust fluids, t_s log-spaced 1e-3..10, eps 0.01 each, "
                       f"g = 0.05, periodic {n}^3, IMEX2P+PLM+HLLE/Rusanov, CFL 0.3, seed {seed}",
           "value": round(value, 2), "unit": "Mzone-cycles/s", "dtype": "f64", "steps": steps,
           "ms_per_step": round(el * 1e3 / steps, 4),
           "roofline": kernel_roofline(times, DUST_KERNEL_ALGO, ncell, f"dust{n}_fp64", DUST_STAGE_BYTES),
           "step_hbm_roofline": {"algo_bytes_per_zone_cycle": DUST_STEP_ALGO_BYTES,
                                 "frac": round(value * 1e6 * DUST_STEP_ALGO_BYTES
                                               / (HBM_PEAK_GBS * 1e9), 4)},
           "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in sorted(times.items())}}
    if not fp32:
        return out
    print("[bench] dust leg, FP32 form", file=sys.stderr, flush=True)
    sim = Sim((n, n, n), physics=physics, scheme=dict(scheme, prec="fp32_bulk"))
    sim.set_state(state)
    el, times, _, _ = timed_run(sim, steps, warmup, list(warm) + list(dts))
    nf = 4 * (len(ts) + 1)
    got = sim.state(device=True).reshape(nf, -1)
    sim.close()
    ref = ref.reshape(nf, -1)
    dust_rho = list(range(4, nf, 4))
    rows = {"rho_gas": [0], "M_gas": [1, 2, 3], "rho_dust": dust_rho,
            "M_dust": [r + a for r in dust_rho for a in (1, 2, 3)]}
    l1 = {k: float((got[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for k, v in rows.items()}
    v32 = ncell * steps / el / 1e6
    out["fp32"] = {"value": round(v32, 2), "unit": "Mzone-cycles/s",
                   "ms_per_step": round(el * 1e3 / steps, 4), "dtype": "f32 (drag solve in f64)",
                   "l1_rel_vs_fp64": {k: float(f"{v:.3e}") for k, v in l1.items()},
                   "compared_after_steps": len(warm) + steps,
                   "roofline": kernel_roofline(times, DUST_KERNEL_ALGO_FP32, ncell, f"dust{n}_fp32",
                                               DUST_STAGE_BYTES_FP32),
                   "step_hbm_roofline": {"algo_bytes_per_zone_cycle": DUST_STEP_ALGO_BYTES // 2,
                                         "frac": round(v32 * 1e6 * (DUST_STEP_ALGO_BYTES // 2)
                                                       / (HBM_PEAK_GBS * 1e9), 4)},
                   "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in sorted(times.items())}}
    return out


PAPER_TABLE = {"A100 (FP64)": 300.0, "MI250X one GCD (FP64)": 250.0}


def paper_config_leg(shape, steps: int, warmup: int, precisions=("fp64", "fp32_bulk"), blocks: bool = True):
    """The scheme and box of the paper's performance table: oblique linear fast wave,
    RK2 + PLM + HLLE + CT, one block of shape cells; the paper's FP64 numbers on other
    hardware are quoted as context."""
    from paper_2608_14048_amd import Sim
    from paper_2608_14048_amd import inputs as I

    print(f"[bench] paper-configuration leg {shape}", file=sys.stderr, flush=True)
    state, _ = I.linear_wave(amp=1e-6, along="box", shape=shape)
    length = (shape[0] / shape[2], shape[1] / shape[2], 1.0)
    ncell = shape[0] * shape[1] * shape[2]
    out = {"workload": f"oblique linear fast wave, {shape[0]}x{shape[1]}x{shape[2]} "
                       "periodic box, RK2+PLM+HLLE+CT, CFL 0.3, one block",
           "paper_mzcps_context": PAPER_TABLE}
    ref, seq = None, None
    for prec in precisions:
        sim = Sim(shape, length, scheme=dict(recon="plm", riemann="hlle", integ="rk2",
                                             courant=0.3, prec=prec))
        sim.set_state(state)
        # the FP32-bulk run takes the FP64 run's dt sequence, so the two end states compare
        el, times, warm, dts = timed_run(sim, steps, warmup, seq)
        got = sim.state(device=True)
        sim.close()
        out[prec] = {"value": round(ncell * steps / el / 1e6, 2), "unit": "Mzone-cycles/s",
                     "steps": steps, "ms_per_step": round(el * 1e3 / steps, 4),
                     "kernel_ms_per_step": {k: round(v[0] / steps, 4)
                                            for k, v in sorted(times.items())}}
        if ref is None:
            ref, seq = got, list(warm) + list(dts)
        else:
            # the wave is a 1e-6 perturbation: measure the error on the perturbation, against
            # the FP64 GPU run (which matches the oracle to 1e-12 per step)
            base, _ = I.linear_wave(amp=0.0, along="box", shape=shape)
            out[prec]["l1_rel_vs_fp64"] = l1_classes(got, ref, base)
            out[prec]["l1_reference"] = (f"the FP64 run on the same dt sequence after {len(seq)} steps; "
                                         "relative to the L1 norm of the wave's perturbation")
        del got
    if blocks and "fp64" in out and all(v % 128 == 0 for v in shape):
        out["fp64_128cube_blocks"] = paper_blocks_run(shape, length, state, seq, steps, warmup, ref)
    return out


def paper_blocks_run(shape, length, state, seq, steps: int, warmup: int, ref):
    """The same box and FP64 scheme as the paper runs it: tiled into 128^3 blocks, each
    padded with 3 ghost layers (PLM + CT) that a device exchange refills after every
    stage.  Each step takes the domain's CFL step from the device (no host round trip);
    it is checked to be the one-block run's dt sequence, and the end state to be the
    one-block run's."""
    import torch

    from paper_2608_14048_amd import Domain

    print("[bench] paper-configuration leg, 128^3 blocks", file=sys.stderr, flush=True)
    block = (128, 128, 128)
    dom = Domain(shape, block, length, ghost=3,
                 scheme=dict(recon="plm", riemann="hlle", integ="rk2", courant=0.3))
    dom.set_state(state)
    dom.batch.tune(2)  # the batch autotuner picks the tile shape of the padded blocks
    same_dt = dom.dt_cfl() == seq[0]
    for k in range(warmup):
        dom.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        dom.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    got = dom.state(device=True)
    nblocks = dom.batch.nb
    shape_used = ("64-wide", "32-wide", "16-wide")[dom.batch.tile_shapes()[0]]
    padded = nblocks * (block[0] + 6) * (block[1] + 6) * (block[2] + 6)
    dom.close()
    ncell = shape[0] * shape[1] * shape[2]
    same = bool(same_dt and torch.equal(got, ref))
    del got
    return {"value": round(ncell * steps / el / 1e6, 2), "unit": "Mzone-cycles/s", "steps": steps,
            "ms_per_step": round(el * 1e3 / steps, 4), "blocks": nblocks, "block_cells": list(block),
            "ghost_layers": 3, "stored_cells_over_domain": round(padded / ncell, 4), "tile_shape": shape_used,
            "bitwise_equal_to_one_block": same,
            "note": "every stage is followed by the ghost exchange; the rate counts domain cells only"}


def l1_classes_blocks(got, ref, shapes):
    """l1_classes over a batch state (the blocks' canonical states one after another)."""
    rows = {"rho": [0], "M": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    num = {k: 0.0 for k in rows}
    den = {k: 0.0 for k in rows}
    at = 0
    for sh in shapes:
        m = int(sh[0] * sh[1] * sh[2])
        g = got[at:at + 8 * m].reshape(8, m)
        r = ref[at:at + 8 * m].reshape(8, m)
        for k, v in rows.items():
            num[k] += float((g[v] - r[v]).abs().sum())
            den[k] += float(r[v].abs().sum())
        at += 8 * m
    return {k: float(f"{num[k] / den[k]:.3e}") for k in rows}


def l1_classes(got, ref, base=None):
    """Relative L1 difference of each MHD conserved class (rho, M, E, B) between two
    device states; with base, relative to the L1 norm of ref - base (a perturbation)."""
    import torch

    g, r = got.reshape(8, -1), ref.reshape(8, -1)
    b = None if base is None else torch.as_tensor(base, device=r.device).reshape(8, -1)
    rows = {"rho": [0], "M": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    out = {}
    for k, v in rows.items():
        den = (r[v] - b[v]).abs().sum() if b is not None else r[v].abs().sum()
        out[k] = float(f"{float((g[v] - r[v]).abs().sum() / den):.3e}")
    return out


def batch_leg(nblocks: int, steps: int, warmup: int, prec: str = "fp32_bulk", seed: int = 0):
    """Batched uneven meshblocks: nblocks self-periodic blocks, each edge uniform in
    {16, 24, 32, 48, 64} (seed), the turbulence recipe per block, VL2+PPM+HLLD+CT.
    The batch (persistent launches, autotuned tile shapes) against the same blocks as
    separate contexts (one launch sequence per block).  Both advance every block by its
    own time step, fixed from the initial state, handed over from the host."""
    import torch

    from paper_2608_14048_amd import Batch, Sim
    from paper_2608_14048_amd import inputs as I

    print(f"[bench] batch leg: {nblocks} blocks ({prec})", file=sys.stderr, flush=True)
    shapes = I.meshblock_shapes(nblocks, seed=seed)
    states = [I.turbulence_block(sh, seed=1000 + b)[0] for b, sh in enumerate(shapes)]
    ncell = int(sum(a * b * c for a, b, c in shapes))
    scheme = dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3, prec=prec)
    bt = Batch(shapes, scheme=scheme)
    bt.set_state(states)
    dts = bt.dt_cfl()
    default_shapes = bt.tile_shapes()
    tune_ms = bt.tune(reps=3)
    chosen = bt.tile_shapes()

    def run_batch():
        for _ in range(warmup):
            bt.step(dts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bt.step(dts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    bt.set_state(states)
    el_tuned = run_batch()
    got32 = bt.state(device=True)
    bt.set_tile_shapes(default_shapes)
    bt.set_state(states)
    el_default = run_batch()
    bt.close()
    del bt
    # the same blocks and time steps in FP64 (default shapes): the reference of the
    # FP32-bulk batch's error
    l1 = None
    if prec == "fp32_bulk" and got32 is not None:
        b64 = Batch(shapes, scheme=dict(scheme, prec="fp64"))
        b64.set_state(states)
        for _ in range(warmup + steps):
            b64.step(dts)
        l1 = l1_classes_blocks(got32, b64.state(device=True), shapes)
        b64.close()
        del b64
    sims = []
    for sh, st in zip(shapes, states):
        sim = Sim(sh, tuple(v / max(sh) for v in sh), scheme=scheme)
        sim.set_state(st)
        sims.append(sim)
    for _ in range(warmup):
        for sim, dt in zip(sims, dts):
            sim.step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for sim, dt in zip(sims, dts):
            sim.step(dt)
    torch.cuda.synchronize()
    el_sep = time.perf_counter() - t0
    for sim in sims:
        sim.close()
    mz = lambda el: round(ncell * steps / el / 1e6, 2)
    classes = sorted(set(sh[0] for sh in shapes))
    return {"workload": f"{nblocks} self-periodic blocks, edges uniform in {{16,24,32,48,64}} (seed {seed}), "
                        f"{ncell / 1e6:.2f} M cells, turbulence per block, VL2+PPM+HLLD+CT, CFL 0.3",
            "dtype": "f32 (E in f64)" if prec == "fp32_bulk" else "f64", "steps": steps,
            "value": mz(el_tuned), "unit": "Mzone-cycles/s", "ms_per_step": round(el_tuned * 1e3 / steps, 4),
            "default_shapes_value": mz(el_default),
            "separate_launches_value": mz(el_sep),
            "separate_launches_ms_per_step": round(el_sep * 1e3 / steps, 4),
            "speedup_vs_separate": round(el_sep / el_tuned, 2),
            "l1_rel_vs_fp64": l1,
            "l1_reference": f"the same {nblocks} blocks in FP64 on the same dt sequence after {warmup + steps} steps",
            "tuned_shape_per_x_extent": {str(x): int(chosen[[sh[0] for sh in shapes].index(x)]) for x in classes},
            "fastest_alone_per_x_extent": {str(x): int(np.argmin(tune_ms[q])) for q, x in enumerate(classes)},
            "tune_ms_per_pass": {str(x): [round(float(v), 4) for v in tune_ms[q]] for q, x in enumerate(classes)}}


CLOSURE_WEIGHTS = os.path.join(ROOT, "paper_2608_14048_amd", "data", "closure_64.npz")


def closure_leg(seeds=(900, 901), steps: int = 8):
    """The learned closure on held-out seeds: 64^3 plain, 64^3 + closure and plain 128^3,
    each against the 256^3 fine run filtered to 64^3 after every step (same dt
    sequence), with the time per coarse step of each."""
    import torch

    from paper_2608_14048_amd import learned as LC

    print("[bench] closure leg", file=sys.stderr, flush=True)
    if not os.path.exists(CLOSURE_WEIGHTS):
        return {"skipped": "no trained weights"}
    cl, meta = LC.load(CLOSURE_WEIGHTS)
    res, times = LC.evaluate(cl, list(seeds), meta["nc"], meta["r"], steps)
    cl.close()
    nc = meta["nc"]
    summ = LC.summary(res)
    mz = lambda ms: round(nc ** 3 / (ms * 1e-3) / 1e6, 2)
    return {"workload": f"decaying turbulence, 64^3 coarse vs 256^3 fine filtered to 64^3, held-out seeds "
                        f"{list(seeds)}, {steps} coarse steps, VL2+PPM+HLLD+CT FP64",
            "l1_rel_after_steps": summ,
            "apriori_loss_trained_vs_plain": [meta.get("heldout_trained_loss"), meta.get("heldout_zero_loss")],
            "ms_per_coarse_step": {k: round(v, 4) for k, v in times.items()},
            "coarse_mzcps": {"plain": mz(times["plain_ms"]), "closure": mz(times["closure_ms"]),
                             "plain_2x": mz(times["plain_2x_ms"])}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(n: int, state, max_seconds: float):
    """Steps of the oracle on the n^3 turbulence workload from `state` until about
    max_seconds have passed (at least one); returns (Mzone-cycles/s, steps, seconds)."""
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
    return n ** 3 * steps / el / 1e6, steps, el


def cpu_baseline(n: int, state, max_seconds: float = 30.0, seed: int = 0):
    """The oracle as it stands on bounded samples: all threads on as many steps of the
    same n^3 workload as fit in about max_seconds, then one thread on the same recipe at
    64^3 for about a third of that (one 256^3 step takes a single core about 40 s)."""
    import oracle

    from paper_2608_14048_amd import inputs as I

    threads = oracle.num_threads()
    value, steps, el = oracle_rate(n, state, max_seconds)
    n1 = 64
    oracle.set_num_threads(1)
    try:
        v1, s1, e1 = oracle_rate(n1, I.turbulence(n1, seed=seed), max_seconds / 3.0)
    finally:
        oracle.set_num_threads(threads)
    return {"value": round(value, 4), "unit": "Mzone-cycles/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{steps} step(s) of the {n}^3 workload from the same initial state "
                      f"({el:.1f} s, {threads} OpenMP threads over k-planes)",
            "single_thread": {"value": round(v1, 4), "unit": "Mzone-cycles/s", "cores": 1,
                              "sample": f"{s1} step(s) of the same recipe at {n1}^3 (seed {seed}), "
                                        f"{e1:.1f} s on one thread"}}


def fp32_leg(n, state, warm_dts, dts, ref64):
    """The FP32-bulk form (FP64 total energy) on the same workload and the same dt
    sequence as the FP64 run (each step still reads its own CFL step, as in the FP64
    loop); reports its throughput and the relative L1 difference of each conserved
    class to the FP64 state after the same steps."""
    from paper_2608_14048_amd import Sim

    print("[bench] FP32-bulk leg", file=sys.stderr, flush=True)
    sim = Sim((n, n, n), scheme=dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3,
                                     prec="fp32_bulk"))
    sim.set_state(state)
    el, times, _, _ = timed_run(sim, len(dts), len(warm_dts), list(warm_dts) + list(dts))
    got = sim.state(device=True).reshape(8, -1)
    ref = ref64.reshape(8, -1)
    rows = {"rho": [0], "M": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
    l1 = {k: float((got[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for k, v in rows.items()}
    sim.close()
    steps = len(dts)
    value = n ** 3 * steps / el / 1e6
    return {"value": round(value, 2), "unit": "Mzone-cycles/s",
            "ms_per_step": round(el * 1e3 / steps, 4), "dtype": "f32 (E in f64)",
            "l1_rel_vs_fp64": {k: float(f"{v:.3e}") for k, v in l1.items()},
            "compared_after_steps": len(warm_dts) + steps,
            "roofline": kernel_roofline(times, KERNEL_ALGO_FP32, n ** 3, f"turb{n}_fp32_bulk",
                                        STAGE_ALGO_BYTES_FP32),
            "step_hbm_roofline": {"algo_bytes_per_zone_cycle": STEP_ALGO_BYTES_FP32,
                                  "frac": round(value * 1e6 * STEP_ALGO_BYTES_FP32 / (HBM_PEAK_GBS * 1e9), 4)},
            "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in sorted(times.items())}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 legs")
    ap.add_argument("--no-dust", action="store_true", help="skip the gas + dust leg")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip the RK2+PLM+HLLE linear-wave leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-meshblock leg")
    ap.add_argument("--no-paper-blocks", action="store_true",
                    help="skip the paper box as coupled 128^3 blocks (the one-block runs stay)")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg")
    ap.add_argument("--batch-blocks", type=int, default=512)
    ap.add_argument("--dust-n", type=int, default=192)
    ap.add_argument("--paper-shape", type=int, nargs=3, default=(512, 512, 256))
    ap.add_argument("--side-steps", type=int, default=50)
    ap.add_argument("--side-warmup", type=int, default=5)
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 2 GiB device copy three times (the calibration "
                         "launch for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2608_14048_amd import Sim
    from paper_2608_14048_amd import inputs as I

    copy_gbs = None
    if args.copy_probe:
        # 2 GiB read + 2 GiB written per launch; the last two launches are timed
        src = torch.ones(1 << 28, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(2):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        copy_gbs = round(2 * 2 * src.numel() * 8 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
        del src, dst

    n = args.n
    print(f"[bench] building the {n}^3 initial state", file=sys.stderr, flush=True)
    state = I.turbulence(n, seed=args.seed)

    sim = Sim((n, n, n), scheme=dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3))
    sim.set_state(state)
    print(f"[bench] {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr, flush=True)
    elapsed, times, warm_dts, dts = timed_run(sim, args.steps, args.warmup)
    ncell = n ** 3
    value = ncell * args.steps / elapsed / 1e6
    ms_per_step = elapsed * 1e3 / args.steps
    # HBM roofline of the kernel class with the largest device time (its stage's bytes of
    # the fused-step traffic model over its launch time)
    roofline = kernel_roofline(times, KERNEL_ALGO, ncell, f"turb{n}_fp64", STAGE_ALGO_BYTES)
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
                              "frac": round(value * 1e6 * STEP_ALGO_BYTES / (HBM_PEAK_GBS * 1e9), 4),
                              "measured": step_traffic(f"turb{n}_fp64", times, ncell, args.steps,
                                                       STEP_ALGO_BYTES)},
        "kernel_ms_per_step": kernel_ms,
    }
    if copy_gbs is not None:
        out["copy_probe_gbs"] = copy_gbs
    if not args.no_fp32:
        out["fp32_bulk"] = fp32_leg(n, state, warm_dts, dts, sim.state(device=True))
    sim.close()
    if not args.no_dust:
        out["dust"] = dust_leg(args.dust_n, args.side_steps, args.side_warmup, args.seed,
                               fp32=not args.no_fp32)
    if not args.no_paper_config:
        out["paper_config"] = paper_config_leg(tuple(args.paper_shape), args.side_steps,
                                               args.side_warmup, blocks=not args.no_paper_blocks)
    if not args.no_batch:
        out["batch"] = batch_leg(args.batch_blocks, max(args.side_steps // 5, 5), 2, "fp32_bulk", args.seed)
    if not args.no_closure:
        out["closure"] = closure_leg()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, state, args.cpu_seconds, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
