#!/usr/bin/env python3
"""Throughput of the cascaded-biquad filter on one MI355X.

One step = one call of sos_filt over the whole signal: a K = 8 cascade over
2^28 float32 samples (x ~ N(0, 1), pole radius U[0.8, 0.98], seed 0), FP64
arithmetic inside the kernel, input already resident in HBM.  Prints one JSON
line; extra detail (per-solver/N sweep, copy ceiling) goes to stderr and, with
--out, to a JSON file.

The FP64 oracle (test infrastructure) runs only in the CPU leg, which
--no-cpu skips as a whole: the oracle's own timing (`cpu_baseline`) and the
accuracy checks of the headline and of the forms against it.  The filter
itself always runs through the HIP library.
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

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3   # the published figure (packed); unpacked FP32 issues at the FP64 rate


def algorithmic_fma_per_sample(solvers, N, L):
    """The paper's FMA count per sample of the cascade (Tables I and III):
    per PH section 6 + (2 log2 L - 4) / N, per CR section 6 + (L - 1) / N
    (its terminal Toeplitz block); one per section of the list."""
    lg = int(math.log2(L))
    return sum(6.0 + ((2 * lg - 4) if s == "ph" else (L - 1)) / N for s in solvers)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Seconds of back-to-back work before a leg's timed region.  While the host
# builds plans the GPU idles and its clock drops; measured on the training
# step, 0.3 s of work left the first timed configuration 14% slow and 1.0 s
# did not.
CLOCK_WARMUP_S = 1.0


def timed_filter(S, torch, plan, x, y, steps, warmup, warm_s=CLOCK_WARMUP_S):
    """Seconds per step: `steps` back-to-back sos_filt launches between HIP
    events on the launch stream, the plan's workspace (if it needs one)
    allocated once beforehand, after `warm_s` seconds of the same launches
    (the clock warm-up)."""
    stream = torch.cuda.current_stream()
    ws = plan.workspace_size(x.numel())
    wsb = torch.empty(ws, dtype=torch.uint8, device=x.device) if ws else None

    def once():
        _check_call(S, plan, x, y, wsb, stream)

    for _ in range(warmup):
        once()
    torch.cuda.synchronize()
    # bring the clocks up before the timed region
    t_end = time.time() + warm_s
    while time.time() < t_end:
        once()
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        once()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def copy_ceiling(torch, x, y, steps=10):
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / steps
    return 2 * x.numel() * x.element_size() / t / 1e9


def bench_batch(S, W, torch, dev, args):
    """The batched ragged workload: 4096 channels, lengths log-uniform in
    [2^10, 2^22] float32 samples, K ~ U{1..16}, pole radius U[0.5, 0.95],
    channel c drawn with seed c.  The autotuner picks N and the tile cap on
    the real buffers; the chosen launch is captured in a HIP graph and the
    graph replays are timed.  A sample of channels is checked against the
    oracle (one channel at a time)."""
    cfg = W.CONFIGS["batch"]
    e = cfg.extra
    lengths = W.batch_lengths(cfg.channels, e["log2_lo"], e["log2_hi"], cfg.seed)
    Ks = W.batch_sections(cfg.channels, e["K_lo"], e["K_hi"], cfg.seed)
    sos = [W.make_sos(int(Ks[c]), cfg.r_lo, cfg.r_hi, cfg.seed + c) for c in range(cfg.channels)]
    total = int(lengths.sum())
    t = time.time()
    xb = torch.empty(total, dtype=torch.float32, device=dev)
    off = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    # the CPU leg's sample: every other channel, kept on the host as drawn
    kept = {}
    for c in range(cfg.channels):
        x_c = W.make_signal(int(lengths[c]), cfg.seed + c, np.float32)
        xb[off[c]:off[c] + lengths[c]] = torch.from_numpy(x_c).to(dev)
        if not args.no_cpu and c % 2 == 0:
            kept[c] = x_c
    yb = torch.empty_like(xb)
    log("batch: %d channels, %d samples, generated in %.1f s" % (cfg.channels, total, time.time() - t))
    t = time.time()
    best, rows = S.batch_tune(sos, lengths, xb, yb, Ns=(16, 32, 64), Ls=(16, 32, 64), tiles=(0, 8, 16, 32),
                              reps=3)
    log("batch autotune (%.1f s): best N=%d L=%d tile_groups=%d %.3f ms" %
        (time.time() - t, best["N"], best["L"], best["tile_groups"], best["seconds"] * 1e3))
    for r in rows:
        log("  tune N=%2d L=%2d tile_groups=%2d: %.3f ms  %.1f GS/s" %
            (r["N"], r["L"], r["tile_groups"], r["seconds"] * 1e3, total / r["seconds"] / 1e9))
    plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", solver="ph", N=best["N"], L=best["L"])
             for s_ in sos]
    b = S.Batch(plans, lengths, tile_groups=best["tile_groups"])
    stream = torch.cuda.Stream()
    S.filt_batched(b, xb, yb)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        S.filt_batched(b, xb, yb, stream=torch.cuda.current_stream())
    # the same clock warm-up as the other legs
    t_end = time.time() + CLOCK_WARMUP_S
    while time.time() < t_end:
        g.replay()
        torch.cuda.synchronize()
    steps = max(5, args.steps // 2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    with torch.cuda.stream(stream):
        for _ in range(steps):
            g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / steps
    gsps = total / sec / 1e9
    log("batch graph replay: %.3f ms  %.1f GS/s  %.0f GB/s" % (sec * 1e3, gsps, 8.0 * total / sec / 1e9))
    out = {"channels": cfg.channels, "samples": total, "mean_K": float(Ks.mean()), "N": best["N"], "L": best["L"],
           "tile_groups": best["tile_groups"], "ms": sec * 1e3, "GSps": gsps,
           "frac_hbm": 8.0 * total / sec / 1e9 / HBM_PEAK_GBS, "tune": rows}
    if not args.no_cpu:
        import oracle
        # the oracle on the host's cores, one thread per channel at a time
        # (channels are independent), on every other channel of the batch
        cpu = host_cpu()
        threads = max(1, min(16, cpu["available"]))
        chans = sorted(kept)
        t = time.time()
        refs = oracle.sosfilt_batch([kept[c] for c in chans], [sos[c] for c in chans], threads=threads)
        tc = time.time() - t
        m = int(sum(lengths[c] for c in chans))
        out["cpu_baseline"] = {"value": m / tc / 1e9, "unit": "GS/s", "cores": threads, "kind": "oracle",
                               "sample": "every other channel of the batch (%d channels, %d samples), FP64 "
                                         "direct form I, one host thread per channel" % (len(chans), m),
                               "nproc": cpu["nproc"], "cpu_model": cpu["cpu_model"]}
        log("batch oracle: %d channels, %d samples on %d threads in %.2f s (%.2f GS/s)"
            % (len(chans), m, threads, tc, m / tc / 1e9))
        # every channel of that sample against the oracle, element by element
        errs = np.empty(len(chans))
        for i, c in enumerate(chans):
            got = yb[off[c]:off[c] + lengths[c]].cpu().numpy()
            errs[i] = oracle.rel_rms(got, refs[i])
            refs[i] = None
        worst = int(np.argmax(errs))
        out["rel_rms_max_sampled"] = float(errs.max())
        out["rel_rms_median_sampled"] = float(np.median(errs))
        out["checked_channels"] = len(chans)
        out["worst_channel"] = int(chans[worst])
        log("batch: rel_rms over %d channels median %.3e max %.3e (channel %d)"
            % (len(chans), out["rel_rms_median_sampled"], errs.max(), chans[worst]))
        del refs, kept
    del xb, yb
    torch.cuda.empty_cache()
    return out


def forms_summary(extra, plain_gsps):
    """The batched, adjoint and precision forms beside the plain one: each
    one's throughput on its own workload, its ratio to the plain GS/s, and
    its error against the FP64 oracle on sampled channels (null when the
    CPU checks were skipped)."""
    b, g, p = extra["batch"], extra["grad"], extra["precision"]
    out = {
        "batched": {"workload": "4096 channels, lengths log-uniform in [2^10, 2^22] float32, K ~ U{1..16}, "
                                "r U[0.5,0.95]; one graph-replayed launch, autotuned",
                    "GSps": b["GSps"], "vs_plain": b["GSps"] / plain_gsps, "N": b["N"], "L": b.get("L"),
                    "rel_rms_max": b.get("rel_rms_max_sampled"),
                    "checked_channels": b.get("checked_channels"),
                    "cpu_baseline": b.get("cpu_baseline")},
        "adjoint": {"workload": "64 x 2^18 float32, K=8, r U[0.5,0.95]; training step: batched forward that "
                                "fills the adjoint's workspace, then the batched adjoint from it",
                    "GSps": g["GSps"], "vs_plain": g["GSps"] / plain_gsps,
                    "one_call_GSps": g["one_call"]["GSps"],
                    "saved_outputs_GSps": g["saved_outputs"]["GSps"],
                    "gx_rel_rms_max": g.get("gx_rel_rms_max"), "gsos_row_err_max": g.get("gsos_row_err_max")},
        "precision": {"workload": "256 x 2^20 float32, K=8, r U[0.9,0.999]; one batched launch per row",
                      "rows": [dict({"compute": r["compute"], "solver": r["solver"], "GSps": r["GSps"],
                                     "vs_plain": r["GSps"] / plain_gsps, "rel_rms_max": r.get("rel_rms_max"),
                                     "fp32_floor_max": r.get("fp32_floor_max")},
                                    **({"slices": r["slices"]} if "slices" in r else {}))
                               for r in p["rows"]]},
    }
    for f in (out["batched"], out["adjoint"]):
        e = f.get("rel_rms_max", f.get("gx_rel_rms_max"))
        f["within_1e-4"] = None if e is None else bool(e <= 1e-4)
    for r in out["precision"]["rows"]:
        r["within_1e-4"] = None if r["rel_rms_max"] is None else bool(r["rel_rms_max"] <= 1e-4)
    return out


HEADLINE_SOURCES = ("kernels.hpp", "plan.hpp", "plan.cpp", "dispatch.hpp", "sosfilt_api.hip")


def kernel_source_hash():
    """Digest of the sources the single-signal tile kernel and its launch
    are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2607_14054_amd", "csrc")
    for f in HEADLINE_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(N, solver_opt, solvers, n):
    """HBM bytes per launch of the headline kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter's reading for a plain copy of known size), or None when the
    summary does not cover this configuration or the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("source_hash") != kernel_source_hash() or t.get("N") != N
            or t.get("solvers") != solvers or t.get("n") != n):
        return None
    return t.get("bytes_per_launch")


def host_cpu():
    """The host's logical CPU count, the CPUs this process may run on, and
    the CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "available": avail, "cpu_model": model}


SWEEP_NS = (4, 8, 16, 32, 64, 128, 256, 512, 1024)


def bench_sweep(S, torch, sos, x, y, n, steps, ref_dev, full):
    """PH and CR at every N of the paper's sweep (8 .. 1024 blocks per lane
    run, and the narrowest width, 4; L = 16) and at L = 32 and 64 for
    8 <= N <= 64, and the deferred-correction PH at N = 128 .. 1024 (AUTO's
    choice where the runs live in the workspace), on the headline signal
    with FP64 arithmetic.  Each point: time per launch, GS/s, its fraction
    of HBM and of the FP64 vector roofline, and (when the oracle's output is
    given) its relative RMS error against the oracle over the whole signal.
    With `full`, also FP32 arithmetic, the deferred-correction PH at
    N = 16 .. 64 and the scalar and block-filtering variants."""
    cases = [(s_, NN, 16, "f64") for s_ in ("ph", "cr") for NN in SWEEP_NS]
    cases += [(s_, NN, L, "f64") for s_ in ("ph", "cr") for L in (32, 64) for NN in (8, 16, 32, 64)]
    cases += [("phd", NN, 16, "f64") for NN in SWEEP_NS if NN >= 128]
    if full:
        cases += [(s_, NN, 16, "f32") for s_ in ("ph", "cr") for NN in (8, 16, 32, 64)]
        cases += [("phd", NN, 16, "f64") for NN in (16, 32, 64)]
        # comparison points: scalar filtering, block filtering (Toeplitz on MFMA)
        cases += [("scalar", 64, 16, "f64"), ("scalar", 64, 16, "f32"), ("block", 64, 16, "f64"),
                  ("block", 64, 16, "f16"), ("block", 64, 16, "bf16")]
    rows = []
    for solver, NN, L, cd in cases:
        p2 = S.Plan(sos, io_dtype="f32", compute_dtype=cd, solver=solver, N=NN, L=L)
        y.fill_(float("nan"))
        # the points run back to back: a full clock warm-up before the first
        s2 = timed_filter(S, torch, p2, x, y, steps, 2, CLOCK_WARMUP_S if not rows else 0.3)
        i2 = p2.info()
        gbs = 8.0 * n / s2 / 1e9
        row = {"solver": solver, "solvers": sorted(set(i2.solver)), "N": NN, "L": L, "compute": cd,
               "tile": p2.tile(n), "waves_per_simd": i2.waves_per_simd, "ms": s2 * 1e3, "GSps": n / s2 / 1e9,
               "frac_hbm": gbs / HBM_PEAK_GBS}
        if cd == "f64" and solver in ("ph", "cr"):
            fma = algorithmic_fma_per_sample(i2.solver, NN, L)
            row["frac_fp64_alu"] = 2.0 * fma * n / s2 / 1e12 / FP64_VECTOR_PEAK_TFLOPS
        if ref_dev is not None:
            d = y.double() - ref_dev
            row["rel_rms"] = float(torch.sqrt((d * d).sum() / (ref_dev * ref_dev).sum()))
            del d
        rows.append(row)
        log("sweep %-6s N=%4d L=%2d %s: tile=%d occ=%d %.3f ms %.1f GS/s  frac_hbm %.3f%s"
            % (solver, NN, L, cd, row["tile"], i2.waves_per_simd, s2 * 1e3, row["GSps"], row["frac_hbm"],
               "  rel_rms %.2e" % row["rel_rms"] if "rel_rms" in row else ""))
    return rows


def sweep_summary(rows):
    """The sweep's points in the bench line: solver, N, L, GS/s, HBM and
    FP64-ALU fractions and error against the oracle."""
    keep = ("solver", "N", "L", "compute", "GSps", "frac_hbm", "frac_fp64_alu", "rel_rms")
    return [{k: r[k] for k in keep if k in r} for r in rows]


def bench_grad(S, W, torch, dev, args):
    """The adjoint workload: 64 channels x 2^18 float32 samples, K = 8,
    r in [0.5, 0.95], loss sum(y * g) with g ~ N(0, 1) (seed + 2); channel c
    drawn with seed c.  One step is a training step of all channels: the
    batched forward that also fills the adjoint's workspace
    (sos_filt_batched_for_backward) and the batched adjoint from it
    (sos_filt_backward_batched_stored), in the automatic adjoint mode
    (recompute from group checkpoints at K = 8).  For comparison: the same
    step as sos_filt_batched plus the one-call sos_filt_backward_batched,
    and with every section output saved.  A sample of channels is checked
    against the oracle adjoint."""
    cfg = W.CONFIGS["grad"]
    C, n = cfg.channels, cfg.n
    sos = [W.make_sos(cfg.K, cfg.r_lo, cfg.r_hi, cfg.seed + c) for c in range(C)]
    xb = torch.empty(C * n, dtype=torch.float32, device=dev)
    gb = torch.empty_like(xb)
    for c in range(C):
        xb[c * n:(c + 1) * n] = torch.from_numpy(W.make_signal(n, cfg.seed + c, np.float32)).to(dev)
        gb[c * n:(c + 1) * n] = torch.from_numpy(W.grad_seed_signal(n, cfg.seed + c, np.float32)).to(dev)
    yb = torch.empty_like(xb)
    gx = torch.empty_like(xb)
    total = C * n
    out = {"channels": C, "samples": total, "K": cfg.K}
    for mode, two_call, key in (("auto", True, None), ("auto", False, "one_call"), ("save", True, "saved_outputs")):
        plans = [S.Plan(s_, io_dtype="f32", compute_dtype="f64", solver="auto", N=64, adjoint=mode)
                 for s_ in sos]
        b = S.Batch(plans, [n] * C)
        assert b.total == total
        ws = torch.empty(max(b.backward_workspace_size(), 16), dtype=torch.uint8, device=dev)

        def one_pass():
            if two_call:
                S.filt_batched_for_backward(b, xb, yb, workspace=ws)
                return S.filt_backward_batched_stored(b, xb, gb, ws, gx)
            S.filt_batched(b, xb, yb)
            return S.filt_backward_batched(b, xb, gb, gx)

        # a pass is about 0.3 ms: at least 10 of them, so that the first
        # launch's start is a small part of the timed region
        sec = timed(torch, one_pass, max(10, args.steps))
        row = {"ms": sec * 1e3, "GSps": total / sec / 1e9}
        label = "%s, %s" % (mode, "two calls" if two_call else "one call")
        log("grad (%s): %d x %d batched forward+backward %.3f ms  %.1f GS/s"
            % (label, C, n, sec * 1e3, total / sec / 1e9))
        if not args.no_cpu:
            import oracle
            _, gsos, first = one_pass()
            torch.cuda.synchronize()
            g_all = gsos.cpu().numpy()
            worst_x, worst_s = 0.0, 0.0
            for c in (0, C // 2, C - 1):
                x64 = xb[c * n:(c + 1) * n].cpu().numpy().astype(np.float64)
                g64 = gb[c * n:(c + 1) * n].cpu().numpy().astype(np.float64)
                rx, rs = oracle.sosfilt_backward(x64, sos[c], g64)
                worst_x = max(worst_x, oracle.rel_rms(gx[c * n:(c + 1) * n].cpu().numpy(), rx))
                g = g_all[first[c]:first[c] + cfg.K]
                worst_s = max(worst_s, float(np.max(np.abs(g - rs) / np.max(np.abs(rs), axis=1, keepdims=True))))
            row["gx_rel_rms_max"] = worst_x
            row["gsos_row_err_max"] = worst_s
            log("grad (%s): sampled channels gx rel_rms %.2e, gsos row err %.2e" % (label, worst_x, worst_s))
        if key is None:
            out.update(row)
        else:
            out[key] = row
        b.close()
        for p_ in plans:
            p_.close()
    return out


def bench_stream(S, W, torch, dev, args):
    """A ragged stream of requests: each request filters 1-64 channels of
    lengths log-uniform in [2^10, 2^18], each channel with one of 64 cached
    cascades (K ~ U{1..16}, r in [0.5, 0.95]).  Per request: the batch
    schedule, one batched launch and a synchronisation, as a serving loop
    would do, either with a new batch per request or by replanning one
    reserved batch (no allocation, asynchronous upload).  Reports requests/s,
    samples/s and the median and 99th-percentile request latency."""
    rng = np.random.default_rng(9)
    pool = [S.Plan(W.make_sos(int(rng.integers(1, 17)), 0.5, 0.95, 500 + i), io_dtype="f32",
                   compute_dtype="f64", N=16) for i in range(64)]
    reqs = []
    for _ in range(200):
        C = int(rng.integers(1, 65))
        lengths = np.floor(2.0 ** rng.uniform(10, 18, size=C)).astype(np.int64)
        chans = rng.integers(0, 64, size=C)
        reqs.append((lengths, chans))
    cap = int(max(r[0].sum() for r in reqs))
    xb = torch.from_numpy(W.make_signal(cap, 7, np.float32)).to(dev)
    yb = torch.empty_like(xb)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    reuse = S.Batch([pool[0]], [1], max_channels=64, max_samples=cap, max_sections=16)

    def serve_new(lengths, chans):
        b = S.Batch([pool[c] for c in chans], lengths)
        S.filt_batched(b, xb, yb, stream=stream)
        stream.synchronize()

    def serve_replan(lengths, chans):
        reuse.replan([pool[c] for c in chans], lengths, stream=stream)
        S.filt_batched(reuse, xb, yb, stream=stream)
        stream.synchronize()

    out = {"requests": len(reqs), "samples": int(sum(r[0].sum() for r in reqs))}
    for name, serve in (("new_batch", serve_new), ("replan", serve_replan)):
        for r in reqs[:10]:
            serve(*r)
        lat = []
        t_all = time.time()
        for r in reqs:
            t = time.time()
            serve(*r)
            lat.append(time.time() - t)
        wall = time.time() - t_all
        lat = np.array(lat)
        row = {"req_per_s": len(reqs) / wall, "GSps": out["samples"] / wall / 1e9,
               "latency_ms_median": float(np.median(lat) * 1e3),
               "latency_ms_p99": float(np.percentile(lat, 99) * 1e3)}
        out[name] = row
        log("stream (%s): %d requests, %.0f req/s, %.2f GS/s, latency median %.3f ms p99 %.3f ms"
            % (name, len(reqs), row["req_per_s"], row["GSps"], row["latency_ms_median"], row["latency_ms_p99"]))
    return out


def bench_grad_long(S, W, torch, dev, args):
    """The adjoint on one long channel: 2^26 float32 samples, K = 8,
    r in [0.5, 0.95]: one sos_filt_backward per step, in the automatic mode
    (recompute) and with saved outputs; and the training step (forward and
    backward) in the automatic mode, as sos_filt + sos_filt_backward and as
    sos_filt_for_backward + sos_filt_backward_stored."""
    n = 1 << 26
    sos = W.make_sos(8, 0.5, 0.95, 0)
    x = torch.from_numpy(W.make_signal(n, 0, np.float32)).to(dev)
    g = torch.from_numpy(W.grad_seed_signal(n, 0, np.float32)).to(dev)
    gx = torch.empty_like(x)
    y = torch.empty_like(x)
    out = {"samples": n}
    steps = max(3, args.steps // 4)
    for mode in ("auto", "save"):
        plan = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver="auto", N=64, adjoint=mode)
        sec = timed(torch, lambda: S.filt_backward(plan, x, g, gx), steps)
        log("grad-long (%s): 2^26 backward %.3f ms  %.1f GS/s" % (mode, sec * 1e3, n / sec / 1e9))
        row = {"ms": sec * 1e3, "GSps": n / sec / 1e9}
        if mode == "auto":
            out.update(row)
            ws = torch.empty(max(plan.backward_workspace_size(n), 16), dtype=torch.uint8, device=dev)

            def one_call():
                S.filt(plan, x, y)
                S.filt_backward(plan, x, g, gx)

            def two_calls():
                S.filt_for_backward(plan, x, y, workspace=ws)
                S.filt_backward_stored(plan, x, g, ws, gx)

            for name, fn in (("step_one_call", one_call), ("step_two_calls", two_calls)):
                s2 = timed(torch, fn, steps)
                out[name] = {"ms": s2 * 1e3, "GSps": n / s2 / 1e9}
                log("grad-long (auto): 2^26 training step, %s: %.3f ms  %.1f GS/s"
                    % (name.replace("step_", "").replace("_", " "), s2 * 1e3, n / s2 / 1e9))
        else:
            out["saved_outputs"] = row
        plan.close()
    return out


def bench_draws(S, W, torch, dev, args):
    """The headline cascade shape over 16 coefficient draws (seeds 0..15,
    K = 8, r in [0.8, 0.98]) on 2^24 float32 samples each: the kernel's
    relative RMS against the FP64 oracle, and the FP32 floor (a plain
    sequential FP32 cascade) on the same draw."""
    import oracle
    n = 1 << 24
    x_np = W.make_signal(n, 0, np.float32)
    xt = torch.from_numpy(x_np).to(dev)
    rows = []
    for seed in range(16):
        sos = W.make_sos(8, 0.8, 0.98, seed)
        plan = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=args.solver, N=args.N or 64)
        y = S.filt(plan, xt).cpu().numpy()
        ref = oracle.sosfilt(x_np, sos)
        rows.append({"seed": seed, "rel_rms": oracle.rel_rms(y, ref), "max_rel": oracle.max_rel(y, ref),
                     "fp32_floor_rel_rms": oracle.rel_rms(oracle.sosfilt_f32arith(x_np, sos), ref)})
    k = np.array([r["rel_rms"] for r in rows])
    f = np.array([r["fp32_floor_rel_rms"] for r in rows])
    out = {"n": n, "draws": rows, "rel_rms_median": float(np.median(k)), "rel_rms_max": float(k.max()),
           "fp32_floor_median": float(np.median(f)), "fp32_floor_max": float(f.max())}
    log("draws: 16 coefficient draws, 2^24 samples: kernel rel_rms median %.2e max %.2e; "
        "FP32 floor median %.2e max %.2e" % (out["rel_rms_median"], out["rel_rms_max"],
                                              out["fp32_floor_median"], out["fp32_floor_max"]))
    return out


def bench_tiny(S, W, torch, dev, args):
    """The small workload (2^16 float64 samples, K = 8, r in [0.5, 0.95],
    seed 0): cache-resident, so a latency.  Per plan, the median of 50
    single calls each between its own events (launch included), the rate of
    50 back-to-back calls, and the relative RMS against the oracle."""
    c = W.CONFIGS["tiny"]
    sos = W.make_sos(c.K, c.r_lo, c.r_hi, c.seed)
    x_np = W.make_signal(c.n, c.seed, np.float64)
    xt = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(xt)
    ref = None
    if not args.no_cpu:
        import oracle
        ref = oracle.sosfilt(x_np, sos)
    out = {"n": c.n, "rows": []}
    # the specified shape (N = 8, L = 64) first, then 16-lane rows
    for solver, N, L in (("ph", 8, 64), ("cr", 8, 64), ("ph", 8, 16), ("cr", 8, 16), ("ph", 16, 16),
                         ("ph", 32, 16), ("cr", 32, 16)):
        plan = S.Plan(sos, io_dtype="f64", compute_dtype="f64", solver=solver, N=N, L=L)
        S.filt(plan, xt, y)
        torch.cuda.synchronize()
        lat = []
        for _ in range(50):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            S.filt(plan, xt, y)
            e1.record()
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1) * 1e3)
        sec = timed(torch, lambda: S.filt(plan, xt, y), 50)
        row = {"solver": solver, "N": N, "L": L, "latency_us_median": float(np.median(lat)),
               "back_to_back_us": sec * 1e6, "GSps": c.n / sec / 1e9}
        if ref is not None:
            import oracle
            row["rel_rms"] = oracle.rel_rms(y.cpu().numpy(), ref)
        out["rows"].append(row)
        log("tiny %s N=%2d L=%2d: latency median %.1f us, back-to-back %.1f us (%.1f GS/s)%s"
            % (solver, N, L, row["latency_us_median"], row["back_to_back_us"], row["GSps"],
               ", rel_rms %.2e" % row["rel_rms"] if "rel_rms" in row else ""))
    return out


def bench_carry(S, W, torch, dev, args):
    """Single signals whose run-in is long against the tile the device needs
    (K = 8, pole radius U[0.9, 0.999], seed 3, float32 I/O, FP64 arithmetic,
    N = 64): the run-in carry against the exact scan carry, at 2^20, 2^24
    and 2^28 samples.  Both are checked against each other."""
    sos = W.make_sos(8, 0.9, 0.999, 3)
    out = {"rows": []}
    for log2n in (20, 24, 28):
        n = 1 << log2n
        xt = torch.from_numpy(W.make_signal(n, 3, np.float32)).to(dev)
        ys = {}
        for carry in ("runin", "scan"):
            plan = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=args.solver, N=64, carry=carry)
            ws = plan.workspace_size(n)
            wsb = torch.empty(max(ws, 16), dtype=torch.uint8, device=dev)
            y = torch.empty_like(xt)

            def once():
                _check_call(S, plan, xt, y, wsb if ws else None)
            sec = timed(torch, once, max(3, args.steps // 4))
            ys[carry] = y
            row = {"log2n": log2n, "carry": carry, "GSps": n / sec / 1e9, "ms": sec * 1e3,
                   "warm_samples": plan.info().warm_samples, "tile": plan.tile(n), "workspace": ws}
            out["rows"].append(row)
            log("carry %-5s 2^%d: %.3f ms %.1f GS/s (run-in %d samples)" % (carry, log2n, sec * 1e3, n / sec / 1e9,
                                                                             row["warm_samples"]))
        d = (ys["runin"] - ys["scan"]).double()
        out["rows"][-1]["rel_rms_scan_vs_runin"] = float(d.norm() / ys["runin"].double().norm())
        del xt, ys
        torch.cuda.empty_cache()
    return out


def _check_call(S, plan, x, y, wsb, stream=None):
    import ctypes
    rc = S.lib().sos_filt(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
                          ctypes.c_void_p(wsb.data_ptr()) if wsb is not None else None,
                          S._stream_ptr(stream) if stream is not None else None)
    if rc != 0:
        raise RuntimeError("sos_filt: status %d" % rc)


def timed(torch, once, steps):
    """Seconds per call: the clock warm-up (CLOCK_WARMUP_S of the same
    calls), then `steps` calls between events on the current stream."""
    t_end = time.time() + CLOCK_WARMUP_S
    while time.time() < t_end:
        once()
        torch.cuda.synchronize()   # one call in flight: the warm-up ends on time
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        once()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def bench_precision(S, W, torch, dev, args):
    """The precision workload: 256 channels x 2^20 float32 samples, K = 8,
    pole radius U[0.9, 0.999], channel c drawn with seed c.  One batched
    launch per arithmetic type and solver (block filtering included); the relative RMS and max error against the
    FP64 oracle on a sample of channels, with the plain sequential FP32
    cascade's error on the same channels (the FP32 floor)."""
    cfg = W.CONFIGS["precision"]
    C, n = cfg.channels, cfg.n
    sos = [W.make_sos(cfg.K, cfg.r_lo, cfg.r_hi, cfg.seed + c) for c in range(C)]
    xb = torch.empty(C * n, dtype=torch.float32, device=dev)
    for c in range(C):
        xb[c * n:(c + 1) * n] = torch.from_numpy(W.make_signal(n, cfg.seed + c, np.float32)).to(dev)
    pick = [0, 1, C // 3, C // 2, C - 1]
    refs = {}
    if not args.no_cpu:
        import oracle
        for c in pick:
            x_c = xb[c * n:(c + 1) * n].cpu().numpy()
            refs[c] = (oracle.sosfilt(x_c, sos[c]), oracle.sosfilt_f32arith(x_c, sos[c]))
    out = {"channels": C, "samples": C * n, "rows": []}
    rows = [("f64", "auto", 64, 0), ("f64", "ph", 64, 0), ("f32", "ph", 64, 0), ("f32", "cr", 64, 0),
            ("f64", "block", 64, 0)]
    # FP16 / BF16 products: one rounding (1 slice), then error-free slices
    # (the default is 3 for FP16, 4 for BF16)
    rows += [("f16", "block", 64, s_) for s_ in (1, 2, 3, 4)] + [("bf16", "block", 64, s_) for s_ in (1, 2, 3, 4)]
    for compute, solver, N, slices in rows:
        plans = [S.Plan(s_, io_dtype="f32", compute_dtype=compute, solver=solver, N=N, slices=slices)
                 for s_ in sos]
        yb = torch.empty_like(xb)
        b = S.Batch(plans, [n] * C)

        def once():
            S.filt_batched(b, xb, yb)
        sec = timed(torch, once, 10)
        row = {"compute": compute, "solver": solver, "N": N, "GSps": C * n / sec / 1e9}
        if solver == "block" and compute != "f64":
            row["slices"] = plans[0].info().block_slices
        if refs:
            import oracle
            errs = [oracle.rel_rms(yb[c * n:(c + 1) * n].cpu().numpy(), refs[c][0]) for c in pick]
            maxs = [oracle.max_rel(yb[c * n:(c + 1) * n].cpu().numpy(), refs[c][0]) for c in pick]
            floor = [oracle.rel_rms(refs[c][1], refs[c][0]) for c in pick]
            row.update({"rel_rms_max": max(errs), "rel_rms_median": float(np.median(errs)),
                        "max_rel_max": max(maxs), "fp32_floor_max": max(floor)})
        out["rows"].append(row)
        log("precision %s/%s N=%d slices=%s: %.1f GS/s %s" % (compute, solver, N, row.get("slices", "-"),
                                                             row["GSps"],
                                                             {k: v for k, v in row.items()
                                                              if "rel" in k or "floor" in k}))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--solver", default="auto")
    ap.add_argument("--N", type=int, default=0)
    ap.add_argument("--compute", default="f64", choices=("f64", "f32"),
                    help="arithmetic of the main plan (f64, the headline's; f32 for comparison profiles)")
    ap.add_argument("--tile", type=int, default=0, help="groups per tile (0: the library's choice)")
    ap.add_argument("--tile-sweep", action="store_true", help="time the main plan at several tile sizes")
    ap.add_argument("--sweep", action="store_true",
                    help="widen the N sweep with FP32 arithmetic, the deferred PH and the scalar and block "
                         "variants")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the sweep of PH and CR over N = 4 .. 1024 (and L = 32, 64)")
    ap.add_argument("--batch", action="store_true",
                    help="also time the batched ragged workload (4096 channels), autotuned, graph-replayed")
    ap.add_argument("--grad", action="store_true",
                    help="also time the adjoint workload (64 channels x 2^18, forward + backward)")
    ap.add_argument("--stream", action="store_true",
                    help="also time a ragged stream of 1-64-channel requests")
    ap.add_argument("--grad-long", action="store_true",
                    help="also time the adjoint on one long channel (2^26 samples)")
    ap.add_argument("--precision", action="store_true",
                    help="also report the error per arithmetic type on the precision workload")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain copy of the signal (counter calibration)")
    ap.add_argument("--tiny", action="store_true",
                    help="also the small FP64 workload's latency")
    ap.add_argument("--carry", action="store_true",
                    help="also the run-in against the exact scan carry on long-run-in single signals")
    ap.add_argument("--no-draws", action="store_true",
                    help="skip the kernel's and the FP32 floor's error over 16 coefficient draws")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU leg: the oracle's timing and every accuracy check that runs the oracle")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, adjoint and precision forms that the default run reports "
                         "beside the plain one")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the cascade is filtered on a single "
              "MI355X; sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_14054_amd import sosfilt as S
    from paper_2607_14054_amd import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    K = 8
    sos = W.make_sos(K, 0.8, 0.98, 0)
    t = time.time()
    x_np = W.make_signal(n, 0, np.float32)
    log("generated %d samples in %.1f s" % (n, time.time() - t))
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    if args.copy_only:
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy: %d launches of %d bytes read + %d written" % (args.steps, 4 * n, 4 * n))
        return

    N = args.N or 64
    plan = S.Plan(sos, io_dtype="f32", compute_dtype=args.compute, solver=args.solver, N=N,
                  tile_groups=args.tile)
    info = plan.info()
    sec = timed_filter(S, torch, plan, x, y, args.steps, args.warmup)
    gsps = n / sec / 1e9
    achieved = 8.0 * n / sec / 1e9
    # the same launch priced in FP64 vector arithmetic, its measured bound
    fma_ps = algorithmic_fma_per_sample(info.solver, info.N, info.L)
    alu_peak = FP64_VECTOR_PEAK_TFLOPS if args.compute == "f64" else FP32_VECTOR_PEAK_TFLOPS
    alu_tflops = 2.0 * fma_ps * n / sec / 1e12
    log("main: N=%d solvers=%s warm=%d tile=%d waves/SIMD=%d  %.3f ms/step  %.1f GS/s  %.0f GB/s"
        % (N, info.solver, info.warm_samples, plan.tile(n), info.waves_per_simd, sec * 1e3, gsps,
           achieved))
    y_np = y.cpu().numpy()

    extra = {"plan": {"N": info.N, "solver": info.solver, "warm_samples": info.warm_samples,
                      "b0_factored": info.b0_factored}}
    copy_gbs = copy_ceiling(torch, x, torch.empty_like(x))
    extra["copy_GBps"] = copy_gbs
    log("copy ceiling: %.0f GB/s" % copy_gbs)

    # the CPU leg: the oracle's time on the headline signal (one channel: the
    # recursion is sequential, one thread) and the headline's error
    cpu = None
    comparator = None
    accuracy = {}
    ref_dev = None
    if not args.no_cpu:
        import oracle
        hc = host_cpu()
        t = time.time()
        ref = oracle.sosfilt(x_np, sos)
        tc = time.time() - t
        cpu = {"value": n / tc / 1e9, "unit": "GS/s", "cores": 1, "kind": "oracle",
               "sample": "the full 2^%d-sample signal, FP64 direct form I, one thread" % args.log2n,
               "nproc": hc["nproc"], "cpu_model": hc["cpu_model"]}
        accuracy["rel_rms"] = oracle.rel_rms(y_np, ref)
        accuracy["max_rel"] = oracle.max_rel(y_np, ref)
        # the FP32 floor: a plain sequential FP32 cascade on the same draw
        accuracy["fp32_floor_rel_rms"] = oracle.rel_rms(oracle.sosfilt_f32arith(x_np, sos), ref)
        log("oracle: %.2f s (%.1f MS/s); rel_rms=%.3e max_rel=%.3e; FP32 floor %.3e"
            % (tc, n / tc / 1e6, accuracy["rel_rms"], accuracy["max_rel"], accuracy["fp32_floor_rel_rms"]))
        ref_dev = torch.from_numpy(ref).to(dev)
        del ref
        # the paper's CPU comparator, scipy.signal.sosfilt in FP64 on one
        # thread, timed on the first 2^26 samples
        try:
            import scipy.signal as ss
            m = min(n, 1 << 26)
            x64 = x_np[:m].astype(np.float64)
            t = time.time()
            ss.sosfilt(np.asarray(sos, dtype=np.float64), x64)
            tc = time.time() - t
            comparator = {"kind": "scipy.signal.sosfilt", "value": m / tc / 1e9, "unit": "GS/s", "cores": 1,
                          "sample": "the first 2^%d samples as FP64" % (m.bit_length() - 1)}
            log("scipy.signal.sosfilt: %.2f s for %d samples (%.1f MS/s)" % (tc, m, m / tc / 1e6))
        except ImportError:
            comparator = None
    del y_np

    if args.tile_sweep:
        rows = []
        for solver, NN in (("ph", 32), ("ph", 64), ("cr", 64), ("ph", 16)):
            for tg in (16, 24, 32, 48, 64, 96, 128):
                p2 = S.Plan(sos, io_dtype="f32", compute_dtype="f64", solver=solver, N=NN, tile_groups=tg)
                s2 = timed_filter(S, torch, p2, x, y, max(3, args.steps // 2), 2, CLOCK_WARMUP_S if not rows else 0.3)
                rows.append({"solver": solver, "N": NN, "tile_groups": tg, "ms": s2 * 1e3,
                             "GSps": n / s2 / 1e9})
                log("tile %s N=%2d tile_groups=%3d: %.3f ms %.1f GS/s" % (solver, NN, tg, s2 * 1e3, n / s2 / 1e9))
        extra["tile_sweep"] = rows

    # PH and CR over the paper's N sweep (and L = 32, 64), run by default
    sweep = None
    if not args.no_sweep:
        sweep = bench_sweep(S, torch, sos, x, y, n, max(3, args.steps // 4), ref_dev, args.sweep)
        extra["sweep"] = sweep
    del ref_dev

    # the forms the metric reports beside the plain one, run by default
    forms = not args.no_forms and not args.copy_only
    if forms:
        args.batch = args.grad = args.precision = True
    if args.batch or args.grad or args.precision or args.grad_long or args.stream:
        del x, y
        torch.cuda.empty_cache()
    if args.batch:
        extra["batch"] = bench_batch(S, W, torch, dev, args)
    if args.grad:
        extra["grad"] = bench_grad(S, W, torch, dev, args)
    if args.grad_long:
        extra["grad_long"] = bench_grad_long(S, W, torch, dev, args)
    if args.stream:
        extra["stream"] = bench_stream(S, W, torch, dev, args)
    if args.precision:
        extra["precision"] = bench_precision(S, W, torch, dev, args)
    if not args.no_cpu and not args.no_draws:   # an accuracy-only leg: part of the CPU leg
        extra["draws"] = bench_draws(S, W, torch, dev, args)
        d = extra["draws"]
        accuracy["draws"] = {"n": d["n"], "count": len(d["draws"]), "rel_rms_median": d["rel_rms_median"],
                             "rel_rms_max": d["rel_rms_max"], "fp32_floor_median": d["fp32_floor_median"],
                             "fp32_floor_max": d["fp32_floor_max"]}
    if args.carry:
        extra["carry"] = bench_carry(S, W, torch, dev, args)
    if args.tiny:
        extra["tiny"] = bench_tiny(S, W, torch, dev, args)

    line = {
        "metric": "GS/s filtered (K=8, FP32) + % HBM roofline; forms vs plain at <=1e-4 rel RMS",
        "value": gsps,
        "unit": "GS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.compute,
        "data": "synthetic",
        "config": {"workload": "plain cascade, 1 channel x 2^%d float32 samples, K=8, "
                               "pole radius U[0.8,0.98], seed 0" % args.log2n,
                   "io_dtype": "f32", "N": info.N, "L": info.L, "solver": args.solver},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(N, args.solver, info.solver, n)},
        "alu_roofline": {"bound": "alu", "achieved": alu_tflops, "peak": alu_peak,
                         "unit": "TFLOP/s", "frac": alu_tflops / alu_peak,
                         "flop_per_sample": 2.0 * fma_ps},
        "cpu_baseline": cpu,
        "cpu_comparator": comparator,
        "accuracy": accuracy,
    }
    if sweep is not None:
        line["sweep"] = sweep_summary(sweep)
    if forms:
        line["forms"] = forms_summary(extra, gsps)
    print(json.dumps(line), flush=True)
    if args.out:
        extra["line"] = line
        with open(args.out, "w") as f:
            json.dump(extra, f, indent=1)


if __name__ == "__main__":
    main()
