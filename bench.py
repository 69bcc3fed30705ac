"""Benchmark of the kernel-fused SAR Range Doppler Algorithm on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one whole RDA (range compression, corner turn, azimuth FFT, RCMC +
azimuth compression) over the 4096 x 4096 complex64 hyperbolic scene
(512-sample range chirp TBP 200, 1024-pulse aperture with up to 8 cells of
range migration, 8-tap Kaiser-sinc RCMC, 5 point targets, 20 dB noise),
with the raw scene resident in HBM.  Prints one JSON line.

Alongside the headline it times, with HIP events on the stream the kernels
run on: each kernel of the fused pipeline inside the pipeline (events between
the four launches of a step; the slowest kernel carries the roofline figure),
the unfused 3-dispatch comparator, and the FP64 CPU oracle on the host cores
(cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
PAPER_FUSED_MPX = 4096 * 4096 / 0.37 / 1e6   # Apple M1 fused RDA, Table II

# Algorithmic bytes per pixel of each kernel launch (read + write complex64);
# filters and per-bin tables are excluded (they stay in L2).
KERNEL_BYTES_PER_PX = {"range_fused": 16, "corner_turn": 16, "azimuth_fft": 16,
                       "rcmc_azimuth": 16}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(a scene would shard by range lines with an all-to-all corner turn; "
              "see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2604_03585_amd as sar
    from sarsim import config, simulate

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = config("c2")
    sc = simulate(cfg)
    Na, Nr = cfg["Na"], cfg["Nr"]
    px = Na * Nr
    raw = torch.from_numpy(sc.raw).to(dev)
    img = torch.empty((Nr, Na), dtype=torch.complex64, device=dev)
    work = torch.empty((Na, Nr), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, reps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / reps, wall

    plan = sar.Plan(cfg, schedule="fused")
    h = plan.handle

    # ---- the timed region: K whole RDA steps ----
    ms_event, wall = timed(lambda: sar.sar_rda_execute(h, raw, img, work, stream),
                           args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = px / (ms_per_step * 1e-3) / 1e6

    # ---- per-kernel durations inside the pipeline (same stream, HIP events
    # between the four launches of each step: the kernels of sar_rda_execute
    # in the same order, on the same buffers) ----
    A, B = work, img
    names = ["range_fused", "corner_turn", "azimuth_fft", "rcmc_azimuth"]
    calls = [lambda: sar.sar_range_compress(h, raw, A, stream),
             lambda: sar.sar_corner_turn(h, A, B, Na, Nr, stream),
             lambda: sar.sar_azimuth_fft(h, B, A, stream),
             lambda: sar.sar_rcmc_azimuth(h, A, B, stream)]
    reps = args.kernel_reps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
    for _ in range(2):
        for c in calls:
            c()
    torch.cuda.synchronize()
    for r in range(reps):
        ev[r][0].record(stream)
        for i, c in enumerate(calls):
            c()
            ev[r][i + 1].record(stream)
    torch.cuda.synchronize()
    kern = {n: sum(ev[r][i].elapsed_time(ev[r][i + 1]) for r in range(reps)) / reps
            for i, n in enumerate(names)}
    dom = max(kern, key=kern.get)
    dom_bytes = KERNEL_BYTES_PER_PX[dom] * px
    achieved = dom_bytes / (kern[dom] * 1e-3) / 1e9

    # ---- unfused 3-dispatch comparator on the same GPU ----
    uplan = sar.Plan(cfg, schedule="unfused")
    ms_unfused, _ = timed(lambda: sar.sar_rda_execute(uplan.handle, raw, img, work, stream),
                          max(10, args.steps // 4), 2)
    torch.cuda.synchronize()
    plan.close()
    uplan.close()

    design_fused = 64 * px        # range 16 + turn 16 + az FFT 16 + RCMC/az 16
    design_unfused = 128 * px     # range 48 + turn 16 + az FFT 16 + RCMC 16 + xH 16 + IFFT 16
    flops = 2 * Na * 5 * Nr * math.log2(Nr) + 2 * Nr * 5 * Na * math.log2(Na)

    out = {
        "metric": "RDA Mpixel/s at 4096^2 FP32 (fused), % HBM peak",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_FUSED_MPX, 1),
        "vs_baseline_ref": "paper fused RDA 0.37 s for 4096^2 on Apple M1 (Table II), context only",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4096x4096 c64 hyperbolic RDA, 8-tap RCMC, 5 targets, 20 dB",
                   "Na": Na, "Nr": Nr, "range_len": cfg["range_len"],
                   "range_tbp": cfg["range_tbp"], "exposure": cfg["exposure"],
                   "schedule": "fused", "parallelism": "none (1 GPU)"},
        "ms_per_step_event": round(ms_event, 4),
        "design_bytes_per_px": 64,
        "hbm_frac_design": round(design_fused / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "fft_gflops": round(flops / (ms_per_step * 1e-3) / 1e9, 1),
        "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
        "unfused": {"ms_per_step": round(ms_unfused, 4),
                    "value": round(px / (ms_unfused * 1e-3) / 1e6, 1),
                    "design_bytes_per_px": 128,
                    "hbm_frac_design": round(design_unfused / (ms_unfused * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4),
                    "fused_speedup": round(ms_unfused / ms_per_step, 2)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": dom_bytes},
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = O.num_threads()
        t0 = time.perf_counter()
        O.rda(sc.raw, cfg)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(px / t / 1e6, 2), "unit": "Mpixel/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "the full 4096x4096 scene once (FP64 oracle, "
                                         f"compute only, {t:.2f} s)"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
