"""Benchmark of the kernel-fused SAR Range Doppler Algorithm on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-split] [--no-batch] [--no-serve]

A step is one whole RDA (range compression, azimuth FFT, RCMC + azimuth
compression; in the turn-free schedule, whose azimuth kernel reads strips of
azimuth lines straight from the range output, so no corner turn) over the
4096 x 4096 complex64 hyperbolic scene
(512-sample range chirp TBP 200, 1024-pulse aperture with up to 8 cells of
range migration, 8-tap Kaiser-sinc RCMC, 5 point targets, 20 dB noise),
with the raw scene resident in HBM.  Prints one JSON line.  Each timed leg
first runs its work for --settle-ms of wall time (default 100 ms, untimed)
so that the GPU clocks have left their idle state, then W warm-up steps,
then the K timed steps.

The timed steps rotate over three buffer sets (raw scene, workspace,
image; 3 x 384 MiB against the 256 MiB MALL), so that every step reads its
raw scene from HBM as a stream of scenes would; one buffer set reused step
after step and a step after a 512 MiB MALL flush are reported beside it.

Besides the headline it measures, each on the same GPU:
  kernels_ms    each kernel of the headline step (same rotating buffers and
                stream, launched back to back by sar_rda_execute), from HIP
                events that the kernel's own dispatch records at its start
                and end (the slowest kernel carries the roofline figure);
  fused_turned  the same scene through the fused schedule with its corner
                turn (64 B/px), with its kernels, and whether its image
                equals the turn-free one bit for bit;
  hbm_copy_gbs  a plain device copy of one 128 MiB scene buffer (read + write
                bytes per second): the achievable rate for a pass;
  unfused       the 3-dispatch comparator;
  split         the same scene with radix-16 butterflies on MFMA (split
                FP16 / BF16 operands, FP32 accumulation), and with FP32
                arithmetic over FP16 intermediate buffers (fp32_halfstore);
  fft_batched   batched 4096-point line FFTs alone (batch 256 and 4096): FP32,
                FP32 in the split real/imaginary LDS layout, and the split
                precisions, in GFLOPS (the paper's Table I comparison);
  batch         64 scenes of uneven size (LFM, Nr 1024..16384, Na 512..8192)
                in shared launches replayed from a hipGraph, autotuned, vs the
                same scenes run one after another;
  serve         Poisson arrivals of scenes 1024^2 .. 8192 x 16384 from a pool
                of 32 device-resident scenes at 0.7 x the measured capacity,
                admitted under an HBM budget: throughput, p50 / p99 latency
                (FP32, split FP16 and half storage at 64 GiB, FP32 at 16 GiB);
  cpu_baseline  the FP64 CPU oracle on the host cores, on the headline scene;
                its image also gives the accuracy of the FP32 and split
                images (relative L2, PSLR / ISLR / SNR differences).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
PAPER_FUSED_MPX = 4096 * 4096 / 0.37 / 1e6   # Apple M1 fused RDA, Table II

# Algorithmic bytes per pixel of each kernel launch (read + write complex64);
# filters and per-bin tables are excluded (they stay in L2).
KERNEL_BYTES_PER_PX = {"range_fused": 16, "corner_turn": 16, "azimuth_fft": 16,
                       "azimuth_strip_fft": 16, "rcmc_azimuth": 16}
KERNEL_SOURCES = ["rda_kernels.inl", "fft_line.hpp", "mfma_fft.hpp", "rda_part_fp32.hip"]
GiB = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="wall time of untimed steps before the warm-up steps of each "
                         "timed leg (GPU clock ramp)")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fft", action="store_true")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-MALL steps (profiling runs: keeps every "
                         "dispatch of a kernel under the pipeline's cache state)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--copy-check", action="store_true",
                    help="only run a plain 256 MiB device copy 10 times (calibrates the "
                         "HBM byte counters of a profiler run) and exit")
    return ap.parse_args()


def cpu_model() -> str | None:
    """The host CPU's model name (as lscpu reports it), if readable."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_03585_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _recorded(tag: str, kernel: str, profiles_dir: str | None):
    d = profiles_dir or os.path.join(ROOT, "profiles")
    want = kernel_source_hash()
    if not os.path.isdir(d):
        return None
    for name in sorted(os.listdir(d)):
        if not name.endswith((".md", ".txt")):
            continue
        for line in open(os.path.join(d, name)):
            if not line.startswith(tag + ":"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("bench_kernel") == kernel and rec.get("source_sha256") == want:
                return rec
    return None


def recorded_traffic(kernel: str, profiles_dir: str | None = None):
    """HBM bytes per launch from the committed counter summary of ``kernel``
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's counts), if it was
    taken on the current kernel sources; else None."""
    return _recorded("traffic-record", kernel, profiles_dir)


def recorded_issue(kernel: str, profiles_dir: str | None = None):
    """VALU / LDS wave-instruction counts per launch of ``kernel`` from the
    committed SQ counter summary, if taken on the current kernel sources."""
    return _recorded("issue-record", kernel, profiles_dir)


# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 VALU
# instruction occupies its SIMD for 4 cycles without packed FP32, an FP32
# transcendental for 16).
VALU_LANE_INSTR_PEAK = 256 * 4 * 16 * 2.4e9


class Timer:
    """HIP-event timing on one stream.  Before the warm-up calls, `fn` runs
    for `settle_ms` of wall time: the GPU's clocks take ~10-20 ms of
    sustained load to reach their steady state, and a timed region that
    starts earlier measures the ramp (the 4096^2 step runs ~8% slower for its
    first ~100 steps after an idle second)."""

    def __init__(self, torch, stream, settle_ms=0.0):
        self.torch, self.stream, self.settle_ms = torch, stream, settle_ms

    def __call__(self, fn, reps, warm):
        torch = self.torch
        t_end = time.perf_counter() + self.settle_ms * 1e-3
        while time.perf_counter() < t_end:
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(self.stream)
        for _ in range(reps):
            fn()
        e1.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / reps, wall / reps * 1e3


N_SETS = 3   # buffer sets the timed steps rotate through (3 x 384 MiB >> the 256 MiB MALL)
KERNELS = {   # the kernels sar_rda_execute launches for the 4096^2 hyperbolic scene
    "turn_free": ["range_fused", "azimuth_strip_fft", "rcmc_azimuth"],
    "fused": ["range_fused", "corner_turn", "azimuth_fft", "rcmc_azimuth"],
}


def headline(args, torch, sar, cfg, raw, dev):
    Na, Nr = cfg["Na"], cfg["Nr"]
    px = Na * Nr
    # Step i works on buffer set i mod 3 (raw, work, img; the same scene in
    # every raw): a set was last touched two steps (768 MiB of traffic)
    # earlier, so each step reads its raw scene from HBM, as a stream of
    # different scenes would, not from the 256 MiB MALL.
    raws = [raw] + [raw.clone() for _ in range(N_SETS - 1)]
    imgs = [torch.empty((Nr, Na), dtype=torch.complex64, device=dev) for _ in range(N_SETS)]
    works = [torch.empty((Na, Nr), dtype=torch.complex64, device=dev) for _ in range(N_SETS)]
    stream = torch.cuda.current_stream()
    timed = Timer(torch, stream, args.settle_ms)
    plans = {s: sar.Plan(cfg, schedule=s) for s in ("turn_free", "fused")}
    it = [0]

    def stepper(plan):
        h = plan.handle

        def step():
            i = it[0] % N_SETS
            it[0] += 1
            sar.sar_rda_execute(h, raws[i], imgs[i], works[i], stream)
        return step

    def breakdown(plan, names, reps):
        """Per-kernel durations of whole steps: the events of every kernel
        sar_rda_execute launches are recorded by the kernels' own dispatches."""
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in names] for _ in range(reps)]
        for row in ev:                     # create the events before the timed launches
            for a, b in row:
                a.record(stream)
                b.record(stream)
        step = stepper(plan)
        timed(step, 2, 2)                  # clocks settled again, queue drained
        for r in range(reps):
            sar.sar_time_next_launches([a for a, _ in ev[r]], [b for _, b in ev[r]])
            step()
        torch.cuda.synchronize()
        return {n: sum(ev[r][i][0].elapsed_time(ev[r][i][1]) for r in range(reps)) / reps
                for i, n in enumerate(names)}

    # ---- the timed region: K whole RDA steps over rotating buffer sets, in
    # the turn-free schedule (no corner turn; the fastest, and bit-identical
    # to the turned one) ----
    ms_event, ms_wall = timed(stepper(plans["turn_free"]), args.steps, args.warmup)
    torch.cuda.synchronize()
    last = (it[0] - 1) % N_SETS
    images = {"fp32": imgs[last].cpu().numpy()}
    kern = breakdown(plans["turn_free"], KERNELS["turn_free"], args.kernel_reps)

    # ---- the same scene with the corner turn (fused schedule), timed the
    # same way; its image must equal the turn-free one bit for bit ----
    ms_turned, _ = timed(stepper(plans["fused"]), args.steps, args.warmup)
    torch.cuda.synchronize()
    same = bool(np.array_equal(imgs[(it[0] - 1) % N_SETS].cpu().numpy().view(np.uint32),
                               images["fp32"].view(np.uint32)))
    kern_turned = breakdown(plans["fused"], KERNELS["fused"], args.kernel_reps)
    turned = {"ms_per_step": ms_turned, "kernels_ms": kern_turned, "image_equal": same}
    img, work = imgs[0], works[0]
    h = plans["turn_free"].handle

    # ---- context: one buffer set, step after step (the raw scene and the
    # previous step's buffers partly stay in the MALL) ----
    ms_warm, _ = Timer(torch, stream, 30.0)(lambda: sar.sar_rda_execute(h, raw, img, work, stream),
                                            20, 2)

    # ---- cold MALL: 512 MiB written between steps evicts the 256 MiB
    # last-level cache, so every step starts from HBM ----
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    cold = []
    for _ in range(0 if args.no_cold else 20):
        scratch.fill_(1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sar.sar_rda_execute(h, raw, img, work, stream)
        e1.record(stream)
        cold.append((e0, e1))
    torch.cuda.synchronize()
    ms_cold = sorted(a.elapsed_time(b) for a, b in cold)[len(cold) // 2] if cold else None
    del scratch, raws, imgs[1:], works[1:]
    plan = plans["turn_free"]

    # ---- achievable HBM rate: a plain device copy of one scene buffer
    # (the runtime's copy kernel), same size and stream as one pass ----
    ms_copy, _ = timed(lambda: work.copy_(raw), 50, 5)
    copy_gbs = 2.0 * raw.numel() * raw.element_size() / (ms_copy * 1e-3) / 1e9

    # ---- unfused 3-dispatch comparator ----
    uplan = sar.Plan(cfg, schedule="unfused")
    ms_unfused, _ = timed(lambda: sar.sar_rda_execute(uplan.handle, raw, img, work, stream),
                          max(10, args.steps // 4), 2)

    # ---- split precisions (MFMA butterflies) ----
    split = {}
    if not args.no_split:
        for prec in ("split_fp16", "split_bf16"):
            with sar.Plan(cfg, precision=prec) as sp:
                ms, _ = timed(lambda: sar.sar_rda_execute(sp.handle, raw, img, work, stream),
                              max(10, args.steps // 2), 3)
                images[prec] = img.cpu().numpy()
            split[prec] = {"ms_per_step": round(ms, 4), "value": round(px / (ms * 1e-3) / 1e6, 1)}
        # FP32 arithmetic with FP16 intermediate buffers (one exponent per line)
        with sar.Plan(cfg, precision="fp32_halfstore") as hp:
            hwork = torch.empty((hp.workspace_bytes + 7) // 8, dtype=torch.complex64, device=dev)
            ms, _ = timed(lambda: sar.sar_rda_execute(hp.handle, raw, img, hwork, stream),
                          max(10, args.steps // 2), 3)
            images["fp32_halfstore"] = img.cpu().numpy()
            del hwork
        split["fp32_halfstore"] = {
            "ms_per_step": round(ms, 4), "value": round(px / (ms * 1e-3) / 1e6, 1),
            "design_bytes_per_px": 40,
            "hbm_frac_design": round(40 * px / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    torch.cuda.synchronize()
    for p in plans.values():
        p.close()
    uplan.close()
    return ms_event, ms_wall, ms_warm, ms_cold, kern, turned, copy_gbs, ms_unfused, split, images


def fft_leg(torch, sar, dev):
    """Batched line FFTs alone (the paper's Table I setting: N = 4096, batch
    256; also batch 4096): GFLOPS at 5 N log2 N per transform for the three
    kernels of that table's comparison: FP32 radix-16 Stockham exchanging
    complex pairs through LDS, the same FP32 butterflies with the split
    real/imaginary LDS layout (forward variant 2), and the split FP16 / BF16
    MFMA butterflies (which need that layout)."""
    import tempfile
    from sarsim import lfm_scene
    s = torch.cuda.current_stream()
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    out = {"n": 4096, "flops_per_fft": 5 * 4096 * 12}
    legs = [("fp32", "fp32", 0), ("fp32_split_layout", "fp32", 2),
            ("split_fp16", "split_fp16", 0), ("split_bf16", "split_bf16", 0)]
    with tempfile.TemporaryDirectory() as td:
        for batch in (256, 4096):
            cfg = lfm_scene(4096, batch, 1, 1, "fft")
            a = torch.randn(batch * 4096, dtype=torch.complex64, device=dev)
            b = torch.empty_like(a)
            for name, prec, variant in legs:
                # the plan copies the forward kernel's variant from the tuning table
                path = os.path.join(td, f"{name}.jsonl")
                with open(path, "w") as f:
                    f.write(json.dumps({"arch": arch, "kind": "fwd", "n": 4096, "prec": 0,
                                        "variant": variant}) + "\n")
                sar.sar_tune_load(path)
                with sar.Plan(cfg, precision=prec) as p:
                    ms, _ = Timer(torch, s, 30.0)(
                        lambda: sar.sar_fft_lines(p.handle, 0, 0, a, b, batch, s),
                        200 if batch == 256 else 50, 5)
                out[f"batch{batch}_{name}"] = {
                    "us": round(ms * 1e3, 2),
                    "gflops": round(5 * 4096 * 12 * batch / (ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(16 * 4096 * batch / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    sar.sar_tune_load(None)
    out["paper_context"] = ("Apple M1: radix-8 Stockham 138 GFLOPS, CT MMA 128, CT scalar in the "
                            "split layout 120 (Table I)")
    return out


def batch_leg(torch, sar, dev):
    from sarsim import batch_configs, simulate_many
    cfgs = batch_configs()
    raws = [None] * len(cfgs)

    def upload(i, sc):
        raws[i] = torch.from_numpy(sc.raw).to(dev)

    t0 = time.perf_counter()
    simulate_many(cfgs, workers=min(16, os.cpu_count() or 8), consume=upload)
    log(f"batch: simulated and uploaded {len(cfgs)} scenes in {time.perf_counter() - t0:.1f} s")
    params = [sar.make_params(c) for c in cfgs]
    # autotune every distinct parameter set (process table only, no cache file)
    t0 = time.perf_counter()
    seen = set()
    for c, p in zip(cfgs, params):
        key = (c["Nr"], c["Na"])
        if key not in seen:
            seen.add(key)
            sar.sar_autotune(p, None)
    tuned = {}
    for n in sorted({c["Nr"] for c in cfgs} | {c["Na"] for c in cfgs}):
        tuned[str(n)] = {"fused": sar.sar_tune_variant(0, n, 0),
                         "batch_fused": sar.sar_tune_variant(4, n, 0)}
    log(f"batch: autotuned {len(seen)} parameter sets in {time.perf_counter() - t0:.1f} s")
    px = sum(c["Na"] * c["Nr"] for c in cfgs)
    s = torch.cuda.Stream()
    timed = Timer(torch, s, 50.0)
    b = sar.sar_batch_plan(params, s)
    imgs = [torch.empty((c["Nr"], c["Na"]), dtype=torch.complex64, device=dev) for c in cfgs]
    work = torch.empty(sar.sar_batch_workspace_bytes(b) // 8 + 1, dtype=torch.complex64,
                       device=dev)
    ms_batch, _ = timed(lambda: sar.sar_batch_execute(b, raws, imgs, work, s), 5, 2)
    # the same batched launches issued directly on the null stream (no graph)
    s0 = torch.cuda.default_stream()
    ms_direct, _ = Timer(torch, s0, 50.0)(lambda: sar.sar_batch_execute(b, raws, imgs, work, 0),
                                          5, 2)
    # the same scenes one after another, one plan each, same stream
    # per scene the schedule the batch gives it: large scenes that the
    # turn-free kernels cover run them (bit-identical; no corner turn)
    def own_schedule(c):
        big = c["Na"] * c["Nr"] >= 1 << 22
        return "turn_free" if big and c["Na"] <= 4096 else "fused"

    plans = [sar.Plan(c, stream=s, schedule=own_schedule(c)) for c in cfgs]
    design_bytes = sum((32 if own_schedule(c) == "turn_free" else 48) * c["Na"] * c["Nr"]
                       for c in cfgs)
    torch.cuda.synchronize()

    def sequential():
        for p, r, im in zip(plans, raws, imgs):
            sar.sar_rda_execute(p.handle, r, im, work, s)

    ms_seq, _ = timed(sequential, 3, 1)
    torch.cuda.synchronize()
    for p in plans:
        p.close()
    sar.sar_batch_destroy(b)
    del raws, imgs, work
    torch.cuda.empty_cache()
    return {"scenes": len(cfgs), "mpx": round(px / 1e6, 1),
            "ms_per_batch": round(ms_batch, 3),
            "value": round(px / (ms_batch * 1e-3) / 1e6, 1),
            "sequential_ms": round(ms_seq, 3),
            "sequential_value": round(px / (ms_seq * 1e-3) / 1e6, 1),
            "speedup_vs_sequential": round(ms_seq / ms_batch, 3),
            "direct_ms": round(ms_direct, 3),
            "design_bytes_per_px": round(design_bytes / px, 2),
            "hbm_frac_design": round(design_bytes / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "turn_free_scenes": sum(own_schedule(c) == "turn_free" for c in cfgs),
            "autotuned_variants": tuned,
            "workload": "64 LFM scenes, Nr 1024..16384 x Na 512..8192 (seed 4), 3-9 targets, "
                        "chirps 1/8 of each axis, one hipGraph replay per batch"}


def serve_leg(args, torch, sar, dev):
    import numpy as np

    from paper_2604_03585_amd.server import (GpuExecutor, Server, latency_summary,
                                             release_on_result, replay)
    from sarsim import serve_pool_configs, simulate_many
    cfgs = serve_pool_configs()
    raws = [None] * len(cfgs)

    def upload(i, sc):
        raws[i] = torch.from_numpy(sc.raw).to(dev)

    t0 = time.perf_counter()
    simulate_many(cfgs, workers=min(16, os.cpu_count() or 8), consume=upload)
    torch.cuda.synchronize()
    log(f"serve: pool of {len(cfgs)} scenes ready in {time.perf_counter() - t0:.1f} s")
    out = {"pool": len(cfgs), "slots": 4,
           "workload": "Poisson arrivals, pool of 32 LFM scenes 1024^2..8192x16384 (seed 5), "
                       "5 targets, 20 dB; each request stages its scene into its own buffers"}
    n_req, n_warm = args.serve_requests, 100
    for prec, budget_gib in (("fp32", 64), ("split_fp16", 64), ("fp32_halfstore", 64),
                             ("fp32", 16)):
        ex = GpuExecutor(4, budget_gib * GiB)
        srv = Server(budget_gib * GiB, slots=4, executor=ex, on_result=release_on_result)
        try:
            # warm plans, then capacity: every request submitted at once
            replay(srv, [(c, r, prec) for c, r in zip(cfgs, raws)], [0.0] * len(cfgs))
            rng = np.random.default_rng(5)
            which = rng.integers(0, len(cfgs), size=n_req + n_warm)
            reqs = [(cfgs[w], raws[w], prec) for w in which]
            # capacity: the median of three bursts (one burst's rate swings by
            # several per cent, and the offered rate follows it)
            caps = []
            for b in range(3):
                burst = reqs[100 * b:100 * b + 300]
                _, err_b, wall = replay(srv, burst, [0.0] * len(burst))
                if err_b:
                    raise RuntimeError(f"serve: burst failed: {next(iter(err_b.values()))}")
                caps.append(len(burst) / wall)
            cap_rps = sorted(caps)[1]
            rate = 0.7 * cap_rps
            arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
            res, err, wall = replay(srv, reqs, arrivals)
        finally:
            srv.close()
            ex.close()
        if err:
            raise RuntimeError(f"serve: {len(err)} requests failed: {next(iter(err.values()))}")
        meas = res[n_warm:]
        px = sum(cfgs[w]["Na"] * cfgs[w]["Nr"] for w in which[n_warm:])
        span = max(r.done for r in meas) - min(r.arrival for r in meas)
        summ = latency_summary(meas)
        key = f"{prec}_{budget_gib}GiB"
        out[key] = {"capacity_req_s": round(cap_rps, 1),
                    "capacity_bursts_req_s": [round(c, 1) for c in caps],
                    "offered_req_s": round(rate, 1),
                    "throughput_mpx_s": round(px / span / 1e6, 1),
                    "p50_ms": round(summ["p50_ms"], 3), "p99_ms": round(summ["p99_ms"], 3),
                    "queue_p99_ms": round(summ["queue_p99_ms"], 3),
                    "max_concurrent": srv.max_concurrent,
                    "max_used_gib": round(srv.max_used / GiB, 2), "budget_gib": budget_gib}
        log(f"serve {key}: {out[key]}")
        del srv, ex, res
        torch.cuda.empty_cache()
    return out


def _median_time(fn, runs):
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], out


def cpu_baseline_leg(sc2, cfg2):
    """The FP64 oracle as it stands, on the host cores (compute only; scene
    generation excluded): the 4096^2 headline scene on all threads (median of
    3, the reported value) and on one thread (one run: about 15 s), the 256^2
    LFM scene on all threads and on one (median of 3), and four
    representative scenes of the 64-scene batch (the quartile sizes) on all
    threads, once each.  About 25-30 s of CPU work in total."""
    from oracle import oracle as O
    from sarsim import batch_configs, config, simulate
    threads = O.num_threads()
    px2 = cfg2["Na"] * cfg2["Nr"]
    legs = {}
    t, ref = _median_time(lambda: O.rda(sc2.raw, cfg2), 3)
    legs["c2_all_threads"] = {"s": round(t, 3), "mpx_s": round(px2 / t / 1e6, 2), "runs": 3}
    cfg1 = config("c1")
    sc1 = simulate(cfg1)
    px1 = cfg1["Na"] * cfg1["Nr"]
    t1, _ = _median_time(lambda: O.rda(sc1.raw, cfg1), 3)
    legs["c1_all_threads"] = {"s": round(t1, 4), "mpx_s": round(px1 / t1 / 1e6, 2), "runs": 3}
    cfgs4 = sorted(batch_configs(), key=lambda c: c["Na"] * c["Nr"])
    picks = [cfgs4[int(q * (len(cfgs4) - 1))] for q in (0.25, 0.5, 0.75, 0.9)]
    c4 = []
    for c in picks:
        s4 = simulate(c)
        tt, _ = _median_time(lambda: O.rda(s4.raw, c), 1)
        c4.append({"Na": c["Na"], "Nr": c["Nr"], "s": round(tt, 3),
                   "mpx_s": round(c["Na"] * c["Nr"] / tt / 1e6, 2)})
    legs["c4_scenes_all_threads"] = c4
    O.set_threads(1)
    try:
        t1s, _ = _median_time(lambda: O.rda(sc1.raw, cfg1), 3)
        t2s, _ = _median_time(lambda: O.rda(sc2.raw, cfg2), 1)
    finally:
        O.set_threads(threads)
    legs["c1_one_thread"] = {"s": round(t1s, 4), "mpx_s": round(px1 / t1s / 1e6, 2), "runs": 3}
    legs["c2_one_thread"] = {"s": round(t2s, 3), "mpx_s": round(px2 / t2s / 1e6, 3), "runs": 1}
    return {"value": round(px2 / t / 1e6, 2), "unit": "Mpixel/s", "cores": threads,
            "kind": "oracle",
            "sample": "the 4096x4096 headline scene, median of 3 runs on all threads (FP64 "
                      f"oracle, compute only, {t:.2f} s each); legs: one thread, the 256^2 "
                      "scene, four batch scenes",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "legs": legs}, ref


def accuracy(images, sc, ref, cfg):
    """Per precision: relative L2 against the oracle image and the largest
    PSLR / ISLR / SNR differences over the targets; plus the per-target
    quality of the FP32 image (the analogue of the paper's Table IV)."""
    from oracle import quality as Q
    rep_ref = Q.point_target_report(ref, sc.targets, 64, 64)
    acc = {"targets_fp32": [
        {"cell": list(r["peak"]), **{k: round(float(r[k]), 3) for k in
                                    ("snr_db", "pslr_range", "islr_range", "pslr_azimuth",
                                     "islr_azimuth")}}
        for r in Q.point_target_report(images["fp32"].T, sc.targets, 64, 64)]}
    for prec, im in images.items():
        img = im.T
        rep = Q.point_target_report(img, sc.targets, 64, 64)
        d = {"rel_l2": float(f"{Q.rel_l2(img, ref):.3e}"),
             "peaks_equal": all(a["peak"] == b["peak"] == (t["m"], t["n"])
                                for a, b, t in zip(rep, rep_ref, sc.targets))}
        for k in ("pslr_range", "islr_range", "pslr_azimuth", "islr_azimuth", "snr_db"):
            d["max_abs_d_" + k] = round(max(abs(a[k] - b[k]) for a, b in zip(rep, rep_ref)), 4)
        acc[prec] = d
    return acc


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a scene "
              "would shard by lines, with the corner turn as an all-to-all; batched "
              "and served scenes would shard whole scenes per GPU).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_check:
        n = 256 << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_check": {"bytes_read": n, "bytes_written": n, "launches": 10}}))
        return

    import paper_2604_03585_amd as sar
    from sarsim import config, simulate

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = config("c2")
    sc = simulate(cfg)
    Na, Nr = cfg["Na"], cfg["Nr"]
    px = Na * Nr
    raw = torch.from_numpy(sc.raw).to(dev)

    ms_event, ms_wall, ms_warm, ms_cold, kern, turned, copy_gbs, ms_unfused, split, images = \
        headline(args, torch, sar, cfg, raw, dev)
    log(f"headline: {ms_wall:.4f} ms/step, kernels {kern}, copy {copy_gbs:.0f} GB/s")
    ms_per_step = ms_wall
    value = px / (ms_per_step * 1e-3) / 1e6
    dom = max(kern, key=kern.get)
    dom_bytes = KERNEL_BYTES_PER_PX[dom] * px
    achieved = dom_bytes / (kern[dom] * 1e-3) / 1e9
    trec = recorded_traffic(dom)
    irec = recorded_issue(dom)
    valu_issue = None
    if irec:
        t = kern[dom] * 1e-3
        cycles = 4 * irec["valu_wave_instr"] + 12 * irec["trans_wave_instr"]
        valu_issue = {"bound": "valu_issue", "kernel": dom,
                      "achieved": round(irec["valu_wave_instr"] * 64 / t / 1e12, 2),
                      "peak": round(VALU_LANE_INSTR_PEAK / 1e12, 2),
                      "unit": "T lane-instr/s",
                      "frac": round(cycles * 16 / t / VALU_LANE_INSTR_PEAK, 4),
                      "valu_per_px": round(irec["valu_wave_instr"] * 64 / px, 1),
                      "lds_conflict_ratio": irec["lds_conflict_ratio"],
                      "source": irec["source"]}

    design_tf = 48 * px           # range 16 + strip az FFT 16 + RCMC/az 16
    design_fused = 64 * px        # range 16 + turn 16 + az FFT 16 + RCMC/az 16
    design_unfused = 128 * px     # range 48 + turn 16 + az FFT 16 + RCMC 16 + xH 16 + IFFT 16
    flops = 2 * Na * 5 * Nr * math.log2(Nr) + 2 * Nr * 5 * Na * math.log2(Na)

    out = {
        "metric": "RDA Mpixel/s at 4096^2 FP32 (fused vs unfused, % HBM peak); p99 scene latency",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "paper_context": f"paper fused RDA 0.37 s for 4096^2 on Apple M1 (Table II): "
                         f"{PAPER_FUSED_MPX:.1f} Mpixel/s on other hardware",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4096x4096 c64 hyperbolic RDA, 8-tap RCMC, 5 targets, 20 dB",
                   "Na": Na, "Nr": Nr, "range_len": cfg["range_len"],
                   "range_tbp": cfg["range_tbp"], "exposure": cfg["exposure"],
                   "schedule": "turn_free (fused kernels, no corner turn)",
                   "parallelism": "none (1 GPU)"},
        "clock_settle_ms": args.settle_ms,
        "buffer_sets": N_SETS,
        "ms_per_step_event": round(ms_event, 4),
        "ms_per_step_one_buffer_set": round(ms_warm, 4),
        "ms_per_step_cold_mall": round(ms_cold, 4) if ms_cold is not None else None,
        "design_bytes_per_px": 48,
        "hbm_frac_design": round(design_tf / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        # the step time against the turned path's 64 B/px: 60% of 8 TB/s at
        # 64 B/px is 224 us per 4096^2 step
        "hbm_frac_64B_equivalent": round(design_fused / (ms_per_step * 1e-3) / 1e9
                                         / HBM_PEAK_GBS, 4),
        "fft_gflops": round(flops / (ms_per_step * 1e-3) / 1e9, 1),
        "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
        "fused_turned": {"ms_per_step": round(turned["ms_per_step"], 4),
                         "value": round(px / (turned["ms_per_step"] * 1e-3) / 1e6, 1),
                         "design_bytes_per_px": 64,
                         "hbm_frac_design": round(design_fused / (turned["ms_per_step"] * 1e-3)
                                                  / 1e9 / HBM_PEAK_GBS, 4),
                         "kernels_ms": {k: round(v, 4) for k, v in turned["kernels_ms"].items()},
                         "image_bit_identical_to_turn_free": turned["image_equal"]},
        "hbm_copy_gbs": round(copy_gbs, 1),
        "unfused": {"ms_per_step": round(ms_unfused, 4),
                    "value": round(px / (ms_unfused * 1e-3) / 1e6, 1),
                    "design_bytes_per_px": 128,
                    "hbm_frac_design": round(design_unfused / (ms_unfused * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4),
                    "fused_speedup": round(ms_unfused / ms_per_step, 2)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (trec["fetch_bytes"] + trec["write_bytes"]) if trec else None,
                     "traffic_source": trec["source"] if trec else None,
                     "algorithmic_bytes": dom_bytes,
                     "kernel_us": round(kern[dom] * 1e3, 2)},
    }
    if valu_issue:
        out["valu_issue"] = valu_issue
    if split:
        out["split"] = split

    if not args.no_fft:
        out["fft_batched"] = fft_leg(torch, sar, dev)
        log(f"fft: {out['fft_batched']}")
    if not args.no_batch:
        out["batch"] = batch_leg(torch, sar, dev)
        log(f"batch: {out['batch']}")
    if not args.no_serve:
        out["serve"] = serve_leg(args, torch, sar, dev)
        out["p99_scene_latency_ms"] = out["serve"]["fp32_64GiB"]["p99_ms"]

    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline_leg(sc, cfg)
        out["accuracy_vs_oracle"] = accuracy(images, sc, ref, cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
