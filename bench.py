#!/usr/bin/env python3
"""Throughput of the overlap-save variable-bandwidth filter on one MI355X.

One step = one vbw_filter call over the whole workload (every channel, every
block: gather, forward FFT, HFSO multiply, inverse FFT, discard, store), with
inputs already resident in HBM.  Default workload: 64 channels x 2^20
complex64 samples, N = 1024, hop 768, 16 transition values per edge, every
channel switching bandwidth at block 512.

Prints one JSON line.  `value` is complex output samples per second of wall
time over the K timed calls; `roofline` takes the kernels' launch duration
from HIP events (the kernels' start and end on every other call; around the
K calls for a graph-replayed plan).  The timed calls are the library call
alone: the fixed buffers are checked once (Plan.bind).  Without --warmup,
about 0.15 s of untimed calls come first, so that the timed calls run past
the power-management transient of the first tens of milliseconds.  The
accuracy of the timed output is checked on sampled blocks against the FP64
oracle (reported in dB); the oracle is also timed on the host cores on a
bounded sample (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "complex output samples/s at ≤ −110 dB vs FP64 oracle; % HBM peak"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2406_14116_amd", "csrc")
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(engine: str) -> str:
    src = os.path.join(CSRC, "ols_gemm.hip" if engine == "gemm" else "ols_fft.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def counters_from_profile(kernel: str, workload_key: str, engine: str):
    """HBM bytes per launch and the VALU / MFMA busy fractions measured by
    rocprofv3 counters, if the committed summary was taken on the current
    kernel source: (traffic or None, {"valu_busy": f, "mfma_busy": f})."""
    path = os.path.join(PROFILE_DIR, f"{kernel}_{workload_key}_pmc.md")
    if not os.path.exists(path):
        return None, {}
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_hash(engine):
        return None, {}
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    busy = {}
    for name in ("VALU", "MFMA"):
        b = re.search(name + r" busy = .* = ([0-9.]+)%", text)
        if b:
            busy[name.lower() + "_busy"] = float(b.group(1)) / 100
    return (float(t.group(1)) if t else None), busy


def make_workload(cfg: int, storage: str, real: bool = False):
    from paper_2406_14116_amd import workloads as wl
    cd = "r32" if real else "c64"
    if cfg == 2:
        return wl.config2(), cd
    if cfg == 3:
        return wl.config3(), cd
    if cfg == 5:
        return wl.config5(), cd
    if cfg == 4:
        return wl.config4(storage=storage), storage
    raise SystemExit(f"config {cfg} is not a bench workload (2, 3, 4, 5)")


def workload_key(cfg: int, storage: str, engine: str, real: bool = False, flags: int = 0) -> str:
    return ({2: "fp32_64ch_n1024", 3: "batched_512ch_mixed", 5: "narrow_256ch_n4096",
             4: f"{storage}_256ch_n256"}[cfg] + ("_gemm" if engine == "gemm" else "") + ("_real" if real else "")
            + ("_noprune" if flags & 1 else ""))


def oracle_input(w, ci: int, dtype: str):
    """What the oracle filters: the values the GPU reads for float32 storage
    (exact in float64), the unquantized samples for 16-bit storage (so the
    error is end to end, input and output rounding included)."""
    from paper_2406_14116_amd import workloads as wl
    if dtype == "c64":
        return wl.channel_samples(w, ci, dtype=np.complex64).astype(np.complex128)
    if dtype == "r32":      # real input: the float32 real parts, exactly
        return wl.channel_samples(w, ci, dtype=np.complex64).real.astype(np.complex128)
    return wl.channel_samples(w, ci)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(w, dtype: str, budget_s: float):
    """Time the FP64 oracle on a bounded sample: seeded random blocks of
    channel 0, as many as fit the time budget at the calibrated rate."""
    from oracle import ols
    c = w.channels[0]
    x = oracle_input(w, 0, dtype)
    v = w.v_sets[c.v_key]
    threads = ols.max_threads()
    rng = np.random.default_rng(77)
    cal = rng.integers(0, c.n_blocks(), size=4 * threads)
    t0 = time.perf_counter()
    ols.blocks_hfso(x, c.n, c.hop, v, c.full_schedule(), blocks=cal)
    per_block = (time.perf_counter() - t0) / len(cal)
    nb = int(max(threads, budget_s / max(per_block, 1e-9)))
    blocks = rng.integers(0, c.n_blocks(), size=nb)   # with repeats when nb > blocks
    t0 = time.perf_counter()
    out = ols.blocks_hfso(x, c.n, c.hop, v, c.full_schedule(), blocks=blocks)
    dt = time.perf_counter() - t0
    samples = len(blocks) * c.hop
    return {"value": samples / dt, "unit": "complex samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(blocks)} seeded random blocks of channel 0 (N={c.n}, hop={c.hop}), "
                      f"{samples} output samples in {dt:.1f} s; direct O(N^2) DFT/IDFT in float64, "
                      f"OpenMP over blocks, {threads} threads on {cpu_model()} ({os.cpu_count()} logical CPUs "
                      f"visible)"}, (blocks, out)


def accuracy(w, dtype, ys, oracle_sample, n_channels: int = 4):
    """dB of the timed output against the oracle on sampled blocks."""
    from oracle import ols
    from paper_2406_14116_amd import harness
    rng = np.random.default_rng(5)
    dbs = []
    blocks0, ref0 = oracle_sample
    got = np.concatenate([harness.storage_to_c128(harness.block_slice(ys[0], w.channels[0].hop, b,
                                                                      w.channels[0].length))
                          for b in blocks0])
    want = np.concatenate([r[: min(w.channels[0].hop, w.channels[0].length - b * w.channels[0].hop)]
                           for b, r in zip(blocks0, ref0)])
    dbs.append(ols.error_db(got, want))
    for ci in rng.choice(np.arange(1, len(w.channels)), size=min(n_channels, len(w.channels) - 1),
                         replace=False):
        c = w.channels[int(ci)]
        sw = c.schedule[0][0] if c.schedule else None
        blocks = harness.sample_blocks(c.n_blocks(), rng, sw, n_random=2)
        x = oracle_input(w, int(ci), dtype)
        ref = ols.blocks_hfso(x, c.n, c.hop, w.v_sets[c.v_key], c.full_schedule(), blocks=blocks)
        g = [harness.storage_to_c128(harness.block_slice(ys[int(ci)], c.hop, b, c.length)) for b in blocks]
        want = [r[: len(gg)] for gg, r in zip(g, ref)]
        dbs.append(ols.error_db(np.concatenate(g), np.concatenate(want)))
    return dbs


TUNE_CACHE = os.path.join(ROOT, "paper_2406_14116_amd", "tune_mi355x.txt")
WARMUP_SECONDS = 0.15


def tune_cache_file(arg):
    """(path, note) of the autotuner choice file for the plan: the given
    path, none for '', else a temporary copy of the package's MI355X file."""
    if arg == "":
        return None, ""
    if arg is not None:
        return arg, f" ({arg})"
    import shutil
    import tempfile
    fd, tmp = tempfile.mkstemp(prefix="vbw_tune_", suffix=".txt")
    os.close(fd)
    if os.path.exists(TUNE_CACHE):
        shutil.copyfile(TUNE_CACHE, tmp)
    return tmp, " (paper_2406_14116_amd/tune_mi355x.txt)"


def copy_bandwidth(nbytes: int, steps: int = 10):
    """GB/s of a plain device copy of nbytes (library copy kernel and torch's
    copy), counting read + write bytes like the filter's algorithmic bytes."""
    import torch
    from paper_2406_14116_amd import vbw
    n = nbytes // 8
    x = torch.empty(n, dtype=torch.complex64, device="cuda").normal_()
    y = torch.empty_like(x)
    out = {}
    for name, fn in (("vbw_copy", lambda: vbw.copy(x, y)), ("torch_copy", lambda: y.copy_(x))):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = 2 * n * 8 / (a.elapsed_time(b) / steps * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return out


def bench_stream(args, w, dtype):
    """Streaming throughput: each channel's stream is fed in C calls per step,
    each call a whole number of blocks (the first chunk of the workload's
    channel, reused, so the buffers stay fixed as in a ring-buffered
    application), history and block counters carried on the device."""
    import torch
    from paper_2406_14116_amd import harness, vbw
    from paper_2406_14116_amd import workloads as wl
    C = args.stream_chunks
    chans = []
    for c in w.channels:
        blocks = max(-(-(c.n - c.hop) // c.hop), c.length // c.hop // C)
        chans.append(wl.Channel(n=c.n, hop=c.hop, lv=c.lv, length=blocks * c.hop, k1=c.k1, v_key=c.v_key,
                                schedule=list(c.schedule)))
    ws = wl.Workload(name=w.name, seed=w.seed, config=w.config, channels=chans, v_sets=w.v_sets,
                     storage=w.storage, description=w.description)
    xs = harness.upload_inputs(ws, dtype)
    ys = harness.alloc_outputs(ws, dtype)
    plan = vbw.Plan.from_workload(ws, dtype=dtype, engine=args.engine, flags=args.flags | vbw.STREAM)
    stream = torch.cuda.current_stream()
    run = plan.bind(xs, ys)          # buffers checked once; each call is the library call only
    s = stream.cuda_stream
    if args.warmup is None:
        args.warmup = 3
    for _ in range(args.warmup * C):
        run(s)
    torch.cuda.synchronize()
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    t0 = time.perf_counter()
    ev[0].record(stream)
    for _ in range(args.steps * C):
        run(s)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gpu_ms = ev[0].elapsed_time(ev[1]) / args.steps
    total = ws.total_samples() * C
    bytes_per_sample = 16 if dtype == "c64" else 8
    line = {
        "metric": METRIC, "value": total / (ms_per_step * 1e-3), "unit": "complex samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name + f"+stream{C}", "channels": len(chans), "total_samples": total,
                   "calls_per_step": C, "samples_per_call_per_channel": chans[0].length, "storage": dtype,
                   "engine": args.engine, "variant": plan.query(vbw.Q_VARIANT), "description": w.description},
        "roofline": {"bound": "hbm", "achieved": total * bytes_per_sample / (gpu_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": total * bytes_per_sample / (gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "kernel_ms": gpu_ms / C},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed calls before the K timed ones (default: as many as fill about 0.15 s, at "
                         "least 3: the clocks reach their sustained state only after some tens of ms of load)")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flags", type=int, default=None,
                    help="plan flags (default: AUTOTUNE, the launch shape timed on the caller's buffers in the "
                         "first, untimed call; with GRAPH for config 3, the batched steady state)")
    ap.add_argument("--variant", type=int, default=None,
                    help="fix the plan's launch variant (vbw_plan_set_variant) instead of the default or autotuned one")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner choice file to read and extend (default: a temporary copy of the choices "
                         "kept for MI355X in the package, so that the run takes them without timing and "
                         "writes nothing into the tree; '' for none)")
    ap.add_argument("--engine", choices=("fft", "gemm"), default="fft",
                    help="gemm: matrix-core DFTs (16-bit storage, N = 256: config 4)")
    ap.add_argument("--storage", choices=("f16", "bf16"), default="f16", help="config 4 storage")
    ap.add_argument("--real", action="store_true",
                    help="configs 2, 3, 5 on real float32 input (the real parts of the samples)")
    ap.add_argument("--stream-chunks", type=int, default=0,
                    help="filter every channel as one stream fed in this many calls per step "
                         "(VBW_STREAM; each call a whole number of blocks on fixed buffers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the library's plain copy over the workload's byte count "
                         "(reference for the memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "channels shard across GPUs with no exchange, but that path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_14116_amd import harness, vbw

    if args.flags is None:
        args.flags = vbw.AUTOTUNE | (vbw.GRAPH if args.config == 3 else 0)
    w, dtype = make_workload(args.config, args.storage, args.real)
    log(f"bench: {w.name}: {len(w.channels)} channels, {w.total_samples()} samples, storage {dtype}")
    if args.copy_calibration:
        nbytes = w.total_samples() * (8 if dtype == "c64" else 4)
        x = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda").normal_()
        y = torch.empty_like(x)
        args.warmup = 3 if args.warmup is None else args.warmup
        for _ in range(args.warmup + args.steps):
            vbw.copy(x, y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": nbytes,
                          "launches": args.warmup + args.steps}), flush=True)
        return
    if args.stream_chunks > 1:
        return bench_stream(args, w, dtype)
    t0 = time.perf_counter()
    xs = harness.upload_inputs(w, dtype)
    ys = harness.alloc_outputs(w, dtype)
    log(f"bench: inputs resident in HBM ({time.perf_counter() - t0:.1f} s)")
    cache, cache_note = tune_cache_file(args.tune_cache)
    before = os.path.getsize(cache) if cache and os.path.exists(cache) else 0
    plan = vbw.Plan.from_workload(w, dtype=dtype, engine=args.engine, flags=args.flags, tune_cache=cache)
    if args.variant is not None:
        plan.set_variant(args.variant)
    # a stream of its own (graph replay needs one other than the null stream)
    stream = torch.cuda.Stream()
    # the buffers stay fixed from call to call, so they are checked once and
    # each call below is the library call alone (Plan.filter checks every
    # tensor per call: about 37 us of Python for config 2, 270 us for config 3)
    run = plan.bind(xs, ys)
    torch.cuda.synchronize()

    # untimed calls; the first one autotunes when the plan has no kept choice
    done = 0
    if args.warmup is None:
        t_call = float("inf")
        for _ in range(3):           # one call's time, after the first call's set-up
            t0 = time.perf_counter()
            run(stream)
            torch.cuda.synchronize()
            t_call = min(t_call, time.perf_counter() - t0)
        done = 3
        args.warmup = max(3, int(np.ceil(WARMUP_SECONDS / max(t_call, 1e-6))))
    for _ in range(args.warmup - done):
        run(stream)
    torch.cuda.synchronize()
    if args.flags & vbw.AUTOTUNE and args.variant is None:
        grew = cache and os.path.exists(cache) and os.path.getsize(cache) > before
        cache_note = ("timed in this run's first call" if not cache or grew else "kept choice") + cache_note
    else:
        cache_note = "fixed" if args.variant is not None else "default shape"

    # Launch duration: every other call takes a pair of events that record the
    # filter kernels' own start and end time (vbw_filter_timed).  (Events on
    # every call would lengthen the wall time of the timed region by about 3%:
    # the runtime's handling of each event sits between consecutive launches.)
    # The span from the first timed call's start to the last one's end, per
    # call, adds the dispatch gaps and is reported beside it.  A graph-replayed
    # plan cannot take kernel events; events recorded around each graph launch
    # would time the event handling as well, so it gets one pair around the K
    # calls, and its launch duration is that span per call.
    kernel_events = not (args.flags & vbw.GRAPH)
    timed = set(range(0, args.steps, 2)) if kernel_events else {0, args.steps - 1}
    ev = {i: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for i in timed}
    if kernel_events:
        for a, b in ev.values():   # create the events before they are handed to the library
            a.record(stream)
            b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i not in ev:
            run(stream)
        elif kernel_events:
            run(stream, ev[i][0], ev[i][1])
        else:
            if i == 0:
                ev[i][0].record(stream)
            run(stream)
            if i == args.steps - 1:
                ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    first, last = min(ev), max(ev)
    span_ms = ev[first][0].elapsed_time(ev[last][1]) / (last - first + 1)
    if kernel_events:
        pairs = [a.elapsed_time(b) for a, b in ev.values()]
    else:
        pairs = [span_ms]
    kernel_ms = float(np.mean(pairs))
    log(f"bench: {ms_per_step:.3f} ms/step wall, {kernel_ms:.3f} ms/launch (events), "
        f"{span_ms:.3f} ms/launch over the span")

    total = w.total_samples()
    bytes_per_sample = 16 if dtype == "c64" else 8
    achieved = total * bytes_per_sample / (kernel_ms * 1e-3) / 1e9
    key = workload_key(args.config, dtype, args.engine, args.real, args.flags)
    kernel = "ols_gemm" if args.engine == "gemm" else "ols_fft"
    traffic, busy = counters_from_profile(kernel, key, args.engine)

    copy = copy_bandwidth(total * bytes_per_sample // 2)
    log(f"bench: plain copy of the same bytes: {copy}")

    cpu = None
    sample = None
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        cpu, sample = cpu_baseline(w, dtype, args.cpu_budget)
    dbs = accuracy(w, dtype, ys, sample) if sample is not None else []

    c0 = w.channels[0]
    line = {
        "metric": METRIC,
        "value": total / (ms_per_step * 1e-3),
        "unit": "real samples/s" if dtype == "r32" else "complex samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name + ("+real" if dtype == "r32" else ""), "channels": len(w.channels), "total_samples": total,
                   "total_blocks": plan.query(vbw.Q_TOTAL_BLOCKS),
                   "n": c0.n if args.config != 3 else "mixed", "hop": c0.hop if args.config != 3 else "3N/4",
                   "storage": dtype, "engine": args.engine, "flags": args.flags,
                   "variant": plan.query(vbw.Q_VARIANT), "variants_searched": plan.query(vbw.Q_N_VARIANTS),
                   "variant_from": cache_note,
                   "description": w.description},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, **busy,
                     "kernel_ms": kernel_ms, "kernel_ms_median": float(np.median(pairs)),
                     "span_ms_per_launch": span_ms, "timed_calls": len(pairs) if kernel_events else args.steps,
                     "launch_timing": "kernel start/end events (vbw_filter_timed)" if kernel_events
                                      else "events on the stream around the timed graph launches, per launch",
                     "algorithmic_bytes": total * bytes_per_sample,
                     "copy_gbs": copy, "frac_of_copy": achieved / max(copy.values())},
        "cpu_baseline": cpu,
        "accuracy_db": {"max": max(dbs) if dbs else None,
                        "median": float(np.median(dbs)) if dbs else None,
                        "channels_checked": len(dbs),
                        "versus": "oracle on the stored float32 input" if dtype in ("c64", "r32") else
                                  "oracle on the unquantized input (end to end: input and output rounding)"},
    }
    plan.close()
    if args.tune_cache is None and cache:
        os.unlink(cache)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
