#!/usr/bin/env python3
"""Throughput of the depth-fused LBP face-recognition path on one MI355X.

A step is one pass of the whole path over one batch resident in HBM: fused
depth median + grey/depth LBP + uniform-59 regional histograms + L1 features
for every crop, then FP32 SVM scores against every enrolled identity and the
per-crop argmax.

Default line (the headline): the ragged batch, the largest end-to-end
workload that fits one GPU -- 16,384 face crops with sides 48-256 px (aspect
0.8-1.25), 8x8 proportional cells, 7552-dim features, 1,024 identities. The
feature kernel is the persistent, largest-first launch chosen by the
project's autotuner, replayed from a HIP graph; scoring is the FP32 MFMA GEMM
+ argmax. Extra keys: the uniform batch (4096 crops of 128x128, 256
identities) as `uniform`; the plain unbatched FP32 GPU path as
`plain_gpu_path`; a serving run (16 RGB-D streams at 30 fps, BF16 scoring
against 1,024 identities, 2 s warm-up + 30 s, through the Python loop, the
plain comparator and the native loop) as `latency`; and the CPU
oracle on the host as `cpu_baseline` (single thread and all of the host's
CPU share), which also states the line's accuracy against the oracle.

Prints one JSON line. `roofline` is the dominant kernel of the step, from
HIP events on the stream the kernels run on, over the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_CROPS, SIDE, N_IDENT, GRID = 4096, 128, 256, 8      # uniform batch
RAGGED_CROPS, RAGGED_IDENT = 16384, 1024               # ragged batch
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
ROTATE = 4
PROFILE_DIR = os.path.join(ROOT, "profiles")
CPU_SHARE = 16  # host threads one GPU's share of the host may use
METRIC = "face crops/s (LBP+hist+SVM) vs plain GPU path at stated acc.; p50/p99 latency"


def _parse():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-latency", action="store_true",
                   help="skip the serving run that gives p50/p99 frame latency")
    p.add_argument("--no-uniform", action="store_true", help="skip the uniform-batch extra key")
    p.add_argument("--latency-seconds", type=float, default=30.0)
    p.add_argument("--latency-warmup", type=float, default=2.0)
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="host seconds each CPU-baseline mode runs for (at least one pass)")
    p.add_argument("--plain-sample", type=int, default=512,
                   help="crops the plain unbatched GPU path is timed on")
    p.add_argument("--workload", default="headline",
                   choices=["headline", "uniform", "ragged", "precision", "serving", "resize",
                            "train"],
                   help="headline (default): the ragged batch with every extra key; uniform "
                        "and ragged: one batch alone; precision, serving, resize, train: the "
                        "other workloads")
    p.add_argument("--resize-frames", type=int, default=1024)
    p.add_argument("--train-identities", type=int, default=256)
    p.add_argument("--train-per-identity", type=int, default=20)
    p.add_argument("--precision-rows", type=int, default=131072)
    p.add_argument("--precision-identities", type=int, default=8192)
    p.add_argument("--ragged-crops", type=int, default=RAGGED_CROPS)
    p.add_argument("--launch", default=None,
                   help="ragged batch: fixed feature launch shape persistent,wg_per_cu,"
                        "row_prefetch,sorted (e.g. 1,4,4,1) instead of the autotuner, so a "
                        "profiled run has no tuning trials")
    p.add_argument("--serve-seconds", type=float, default=30.0)
    p.add_argument("--serve-warmup", type=float, default=2.0)
    return p.parse_args()


def _source_digest(paths):
    """Hash of the sources' code: comments and whitespace are dropped, so an
    edit to the documentation does not disown the counters."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "features": ["paper_1504_01883_amd/csrc/features.hip",
                 "paper_1504_01883_amd/csrc/lbpf_internal.h"],
    "score": ["paper_1504_01883_amd/csrc/score.hip",
              "paper_1504_01883_amd/csrc/lbpf_internal.h"],
}


def _traffic(workload: str, kernel: str):
    """Counter-measured HBM bytes per launch from
    profiles/<workload>_<kernel>_traffic.json, or None when absent or taken on
    a different kernel source."""
    path = os.path.join(PROFILE_DIR, f"{workload}_{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_digest") != _source_digest(KERNEL_SOURCES[kernel]):
        return None
    return t.get("bytes_per_launch")


# Wave64 VALU instructions a second over the chip: 1,024 SIMDs at 2.4 GHz, one
# instruction per 4 cycles each (16 lanes a cycle).
VALU_ISSUE_PEAK_GINST = 256 * 4 * 2.4 / 4


def _valu_issue(ms: float, workload: str, kernel: str):
    """The kernel's VALU issue rate against the chip's: SQ_INSTS_VALU per launch
    from profiles/<workload>_<kernel>_valu.json (same source digest rule as the
    traffic), divided by this run's duration; None without a matching file."""
    path = os.path.join(PROFILE_DIR, f"{workload}_{kernel}_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_digest") != _source_digest(KERNEL_SOURCES[kernel]):
        return None
    gi = t["sq_insts_valu_per_dispatch"] / (ms * 1e-3) / 1e9
    return {"insts_per_launch": t["sq_insts_valu_per_dispatch"], "achieved": gi,
            "peak": VALU_ISSUE_PEAK_GINST, "unit": "G wave64 instructions/s",
            "frac": gi / VALU_ISSUE_PEAK_GINST}


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _kernel_entry(ms, bound, work, workload, kernel):
    if bound == "hbm":
        gbs = work / (ms * 1e-3) / 1e9
        return {"ms": ms, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic(workload, kernel),
                "algorithmic_bytes": work, "valu_issue": _valu_issue(ms, workload, kernel)}
    tf = work / (ms * 1e-3) / 1e12
    return {"ms": ms, "bound": "mfma", "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
            "traffic": _traffic(workload, kernel), "algorithmic_flops": work}


def _roofline(kernels):
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    dk = kernels[dom]
    return {"kernel": dom, "bound": dk["bound"], "achieved": dk["achieved"], "peak": dk["peak"],
            "unit": dk["unit"], "frac": dk["frac"], "traffic": dk["traffic"]}


def _timed_steps(step, steps, warmup):
    """Warm-up, then `steps` timed steps with three events each (before the
    features, between features and scoring, after scoring) on the current
    stream. Returns (ms per step, features ms, scoring ms, per-step
    statistics: median and p90 of each step's span and of its two parts)."""
    import torch
    for i in range(warmup):
        step(i, None)
    torch.cuda.synchronize()
    evs = [_events(3) for _ in range(steps)]
    start, end = _events(2)
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        step(i, evs[i])
    end.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / steps
    f = np.array([e[0].elapsed_time(e[1]) for e in evs])
    sc = np.array([e[1].elapsed_time(e[2]) for e in evs])
    stats = {"reps": steps, "step_ms_median": float(np.median(f + sc)),
             "step_ms_p90": float(np.percentile(f + sc, 90)),
             "features_ms_median": float(np.median(f)), "features_ms_p90": float(np.percentile(f, 90)),
             "score_ms_median": float(np.median(sc)), "score_ms_p90": float(np.percentile(sc, 90))}
    return ms_step, float(f.mean()), float(sc.mean()), stats


# --- the ragged batch (headline) -------------------------------------------


def make_ragged_inputs(n, K):
    """Host inputs of the ragged batch (rendered in worker processes, before
    the GPU is touched)."""
    from paper_1504_01883_amd import synth
    t0 = time.time()
    g, z, offs, sizes, labels = synth.make_ragged(n, K, workers=min(CPU_SHARE, os.cpu_count() or 1))
    print(f"[bench] generated {n} ragged crops in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    return g, z, offs, sizes, labels


def run_ragged(args, ctx, host):
    """The ragged step: features of every crop (the tuned persistent kernel,
    replayed from a HIP graph) + FP32 scores and argmax against 1024
    identities (one scoring call). Returns the result dict and the state the
    comparator and CPU legs need."""
    import torch

    from paper_1504_01883_amd import synth, tune
    g, z, offs, sizes, _ = host
    n, K = len(sizes), RAGGED_IDENT
    D = ctx.dim
    dg = torch.from_numpy(g).cuda()
    dz = torch.from_numpy(z.view(np.int16)).cuda()
    planes = []
    for o, (w, h) in zip(offs, sizes):
        o, w, h = int(o), int(w), int(h)
        planes.append((dg[o:o + w * h].view(h, w), dz[o:o + w * h].view(h, w)))
    boxes = [[i, 0, 0, int(w), int(h)] for i, (w, h) in enumerate(sizes)]
    batch = ctx.batch(planes, boxes)
    W, b = synth.synthetic_weights(K, D, synth.W_RAGGED)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda())
    hist = torch.empty((n, D), dtype=torch.float32, device="cuda")
    S = torch.empty((n, K), dtype=torch.float32, device="cuda")
    A = torch.empty((n,), dtype=torch.int32, device="cuda")
    area = float((sizes[:, 0] * sizes[:, 1]).mean())
    if args.launch:
        p, m, pf, so = (int(v) for v in args.launch.split(","))
        batch.set_launch(persistent=p, wg_per_cu=m, row_prefetch=pf, sorted=so)
        tuned = {"cfg": batch.get_launch(), "us": None, "cached": False, "fixed": True}
    else:
        tuned = tune.tuned(ctx, batch, hist, n, area, reps=10, retune=True)
    graph = ctx.graph(batch, hist)  # the feature launch, captured once

    def step(i, ev):
        if ev is not None:
            ev[0].record()
        graph.launch()
        if ev is not None:
            ev[1].record()
        ctx.score(hist, wts, scores_out=S, argmax_out=A)
        if ev is not None:
            ev[2].record()

    ms_step, feat_ms, score_ms, stats = _timed_steps(step, args.steps, args.warmup)
    feat_bytes = float(3 * (sizes[:, 0] * sizes[:, 1]).sum() + n * D * 4)
    score_flops = 2.0 * n * K * D
    kernels = {"features": _kernel_entry(feat_ms, "hbm", feat_bytes, "ragged", "features"),
               "score_fp32": _kernel_entry(score_ms, "mfma", score_flops, "ragged", "score")}

    # The same step with FP32-accurate split FP16 scoring (LBPF_F16X3: three
    # FP16 products on the matrix cores; its accuracy against the FP64 oracle
    # is stated by the CPU leg on the same sample as the FP32 scores').
    wts3 = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="f16x3")
    S3 = torch.empty_like(S)
    A3 = torch.empty_like(A)

    def step3(i, ev):
        if ev is not None:
            ev[0].record()
        graph.launch()
        if ev is not None:
            ev[1].record()
        ctx.score(hist, wts3, scores_out=S3, argmax_out=A3)
        if ev is not None:
            ev[2].record()

    ms3, feat3, score3, _ = _timed_steps(step3, args.steps, args.warmup)
    tf3 = score_flops / (score3 * 1e-3) / 1e12
    split = {"value": n / (ms3 * 1e-3), "unit": "crops/s", "ms_per_step": ms3,
             "features_ms": feat3, "score_ms": score3, "effective_tflops": tf3,
             "mfma_frac": 3 * tf3 / 2500.0, "peak_tflops": 2500.0,
             "note": "scores from FP16 high/low parts of X and W (hi hi + hi lo + lo hi, FP32 "
                     "accumulation, feature-row split + GEMM + argmax in score_ms); mfma_frac "
                     "counts the three FP16 products against the dense FP16 peak"}
    out = {"value": n / (ms_step * 1e-3), "ms_per_step": ms_step,
           "config": {"workload": f"ragged batch: {n} face crops, sides 48-256 px (aspect "
                                  f"0.8-1.25, mean area {area:.0f} px), grey u8 + depth u16, "
                                  f"8x8 proportional cells, {D}-dim uniform-59 features, {K} "
                                  "identities, FP32 scoring + argmax; the tuned persistent "
                                  "feature kernel replayed from a HIP graph",
                      "crops": n, "identities": K, "dim": D, "mean_area": area,
                      "parallelism": "single GPU"},
           "tuned_launch": tuned, "roofline": _roofline(kernels), "kernels": kernels,
           "step_stats": stats, "split_f16_scoring": split}
    state = {"planes": planes, "boxes": boxes, "wts": wts, "W": W, "b": b, "hist": hist,
             "S": S, "A": A, "S3": S3, "A3": A3, "keep": (dg, dz, batch, graph, wts3)}
    return out, state


def plain_ragged(ctx, state, sample):
    """The plain unbatched FP32 GPU path (per-crop launches, global atomics,
    GEMV scoring) on the first `sample` crops of the same resident inputs."""
    import torch
    n = min(sample, len(state["boxes"]))
    planes = state["planes"][:n]
    boxes = state["boxes"][:n]
    wts = state["wts"]
    hist = torch.empty((n, ctx.dim), dtype=torch.float32, device="cuda")
    S = torch.empty((n, wts.K), dtype=torch.float32, device="cuda")
    A = torch.empty((n,), dtype=torch.int32, device="cuda")
    ctx.features_plain(planes[:8], boxes[:8], out=hist[:8])
    ctx.score_plain(hist[:8], wts, scores_out=S[:8], argmax_out=A[:8])
    torch.cuda.synchronize()
    e0, e1 = _events(2)
    e0.record()
    ctx.features_plain(planes, boxes, out=hist)
    ctx.score_plain(hist, wts, scores_out=S, argmax_out=A)
    e1.record()
    torch.cuda.synchronize()
    rate = n / (e0.elapsed_time(e1) * 1e-3)
    return {"value": rate, "unit": "crops/s",
            "sample": f"first {n} crops of the ragged batch, one crop per launch"}


# --- the uniform batch -------------------------------------------------------


def run_uniform(args, ctx, host):
    """The uniform step: one fused feature launch over 4096 crops of 128x128 +
    FP32 scores and argmax against 256 identities; four rotating input and
    output sets (1.3 GB) so the 256 MB last-level cache cannot serve repeats."""
    import torch

    from paper_1504_01883_amd import lbpf, synth
    grey, depth = host
    dev = torch.device("cuda", 0)
    D = ctx.dim
    W, b = synth.synthetic_weights(N_IDENT, D, synth.W_UNIFORM)
    g_host = grey.reshape(N_CROPS * SIDE, SIDE)
    z_host = depth.reshape(N_CROPS * SIDE, SIDE)
    boxes = synth.stacked_boxes(N_CROPS, SIDE, SIDE)
    planes, batches, hists = [], [], []
    for _ in range(ROTATE):
        g, z = lbpf.to_device_planes(g_host, z_host, dev)
        planes.append((g, z))
        batches.append(ctx.batch([(g, z)], boxes))
        hists.append(torch.empty((N_CROPS, D), dtype=torch.float32, device=dev))
    wts = ctx.weights(torch.from_numpy(W).to(dev), torch.from_numpy(b).to(dev))
    scores = torch.empty((N_CROPS, N_IDENT), dtype=torch.float32, device=dev)
    argmax = torch.empty((N_CROPS,), dtype=torch.int32, device=dev)

    def step(i, ev):
        r = i % ROTATE
        if ev is not None:
            ev[0].record()
        ctx.features_batch(batches[r], hists[r])
        if ev is not None:
            ev[1].record()
        ctx.score(hists[r], wts, scores_out=scores, argmax_out=argmax)
        if ev is not None:
            ev[2].record()

    ms_step, feat_ms, score_ms, stats = _timed_steps(step, args.steps, args.warmup)
    feat_bytes = N_CROPS * (SIDE * SIDE * 3 + D * 4)   # grey + depth in, FP32 row out
    score_flops = 2.0 * N_CROPS * N_IDENT * D
    kernels = {"features": _kernel_entry(feat_ms, "hbm", feat_bytes, "uniform", "features"),
               "score_fp32": _kernel_entry(score_ms, "mfma", score_flops, "uniform", "score")}
    out = {"value": N_CROPS / (ms_step * 1e-3), "unit": "crops/s", "ms_per_step": ms_step,
           "config": {"workload": "uniform batch: 4096 face crops 128x128 (grey u8 + depth u16), "
                                  "8x8 grid, 7552-dim uniform-59 features, 256 identities, FP32 "
                                  "scoring + argmax; one fused feature launch + one scoring call",
                      "crops": N_CROPS, "side": SIDE, "identities": N_IDENT, "dim": D},
           "roofline": _roofline(kernels), "kernels": kernels, "step_stats": stats}
    for bt in batches:
        bt.close()
    state = {"W": W, "b": b, "scores": scores, "argmax": argmax, "hist": hists[0],
             "planes": planes, "wts": wts}
    return out, state


def _calibration_copy():
    """A copy of known size for the HBM byte counters: reads and writes
    exactly 256 MiB (an elementwise kernel, visible to the profiler)."""
    import torch
    src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.add(src, 1, out=dst)
    torch.cuda.synchronize()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}); crops are "
              "independent, so the path shards by crop, but no multi-GPU run is implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "resize":
        return bench_resize(args)
    if args.workload == "train":
        return bench_train(args)
    if args.workload == "serving":
        from paper_1504_01883_amd import serve
        print(json.dumps(serve.bench(args)), flush=True)
        return None
    if args.workload == "uniform":
        return bench_uniform(args)

    # Inputs first: the ragged crops are rendered in forked worker processes,
    # which must happen before this process initialises the GPU.
    from paper_1504_01883_amd import synth
    headline = args.workload == "headline"
    host_r = make_ragged_inputs(args.ragged_crops, RAGGED_IDENT)
    host_u = None
    if headline and not args.no_uniform:
        grey, depth, _ = synth.make_crops(N_CROPS, SIDE, SIDE, synth.W_UNIFORM, N_IDENT)
        host_u = (grey, depth)

    import torch

    from paper_1504_01883_amd import lbpf
    torch.cuda.set_device(0)
    ctx = lbpf.Context()
    _calibration_copy()
    res, st = run_ragged(args, ctx, host_r)
    print(f"[bench] ragged: {res['value'] / 1e6:.2f} M crops/s, features "
          f"{res['kernels']['features']['ms'] * 1e3:.0f} us, scoring "
          f"{res['kernels']['score_fp32']['ms'] * 1e3:.0f} us", file=sys.stderr, flush=True)
    out = {"metric": METRIC if headline else "face crops/s (LBP+hist+SVM), ragged batch",
           "value": res["value"], "unit": "crops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": res["config"], "roofline": res["roofline"], "kernels": res["kernels"],
           "tuned_launch": res["tuned_launch"], "step_stats": res["step_stats"],
           "split_f16_scoring": res["split_f16_scoring"]}
    if not headline:
        print(json.dumps(out), flush=True)
        ctx.close()
        return None

    plain = plain_ragged(ctx, st, args.plain_sample)
    plain["fused_speedup"] = res["value"] / plain["value"]
    out["plain_gpu_path"] = plain

    uni = None
    if host_u is not None:
        uni, ust = run_uniform(args, ctx, host_u)
        out["uniform"] = uni
        print(f"[bench] uniform: {uni['value'] / 1e6:.2f} M crops/s", file=sys.stderr, flush=True)

    latency = None
    if not args.no_latency:
        from paper_1504_01883_amd import serve
        latency = serve.quick_latency(ctx, seconds=args.latency_seconds,
                                      warmup=args.latency_warmup, keep_results=True)
        out["latency"] = {k: v for k, v in latency.items() if not k.startswith("_")}
        print(f"[bench] serving: p99 {latency['fused_bf16'].get('p99_ms')} ms (Python loop), "
              f"{latency['fused_bf16_native'].get('p99_ms')} ms (native loop)", file=sys.stderr,
              flush=True)

    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        out["cpu_baseline"] = cpu_baseline(host_r, st, args.cpu_seconds, out, latency)
    print(json.dumps(out), flush=True)
    ctx.close()
    return None


def bench_uniform(args):
    """The uniform batch alone (its own JSON line)."""
    from paper_1504_01883_amd import synth
    grey, depth, _ = synth.make_crops(N_CROPS, SIDE, SIDE, synth.W_UNIFORM, N_IDENT)
    import torch

    from paper_1504_01883_amd import lbpf
    torch.cuda.set_device(0)
    ctx = lbpf.Context()
    _calibration_copy()
    res, _ = run_uniform(args, ctx, (grey, depth))
    out = {"metric": "face crops/s (LBP+hist+SVM), uniform batch", "value": res["value"],
           "unit": "crops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic", "config": res["config"],
           "roofline": res["roofline"], "kernels": res["kernels"]}
    print(json.dumps(out), flush=True)
    ctx.close()


# --- CPU baseline (the oracle) and the stated accuracy ------------------------


def _oracle_pass(oracle, g, z, offs, sizes, idx, W, b, threads):
    imgs = []
    for i in idx:
        o, w, h = int(offs[i]), int(sizes[i][0]), int(sizes[i][1])
        imgs.append((g[o:o + w * h].reshape(h, w), z[o:o + w * h].reshape(h, w)))
    boxes = np.array([[k, 0, 0, int(sizes[i][0]), int(sizes[i][1])] for k, i in enumerate(idx)],
                     np.int32)
    f, _, _ = oracle.features(imgs, boxes, n_threads=threads)
    s64, am = oracle.score_f64(f, W, b, want_scores=True, n_threads=threads)
    return f, s64, am


def _time_mode(oracle, host, st, threads, seconds, first):
    """Oracle passes over a sample of the ragged crops (starting at crop
    `first`), the sample grown until one pass takes a tenth of `seconds`, then
    repeated until `seconds` of host time have run."""
    g, z, offs, sizes, _ = host
    n = len(sizes)
    m = 8 * threads
    while True:
        idx = np.arange(first, first + m) % n
        t0 = time.perf_counter()
        res = _oracle_pass(oracle, g, z, offs, sizes, idx, st["W"], st["b"], threads)
        dt = time.perf_counter() - t0
        if dt >= seconds / 10 or m >= n:
            break
        m = min(n, int(m * max(2.0, seconds / 10 / max(dt, 1e-3))))
    crops, elapsed = m, dt
    while elapsed < seconds:
        t0 = time.perf_counter()
        _oracle_pass(oracle, g, z, offs, sizes, idx, st["W"], st["b"], threads)
        elapsed += time.perf_counter() - t0
        crops += m
    return crops / elapsed, idx, res, elapsed, crops


def cpu_baseline(host, st, seconds, out, latency):
    """The CPU oracle, unchanged, on bounded samples of the ragged batch:
    features + FP64 scores + argmax, once with one thread and once with the
    host's CPU share. The all-thread pass also states the line's accuracy:
    the GPU's FP32 features against the oracle's (bit for bit), its FP32
    scores' largest error relative to the dot product's condition scale and
    its argmax agreement; and, for the serving run, the BF16 scores' largest
    error against the oracle's FP64 scores and their argmax agreement."""
    import oracle
    threads = min(CPU_SHARE, os.cpu_count() or 1)
    r1, _, _, t1, c1 = _time_mode(oracle, host, st, 1, seconds, first=0)
    rn, idx, (f, s64, am), tn, cn = _time_mode(oracle, host, st, threads, seconds, first=0)
    hist = st["hist"][idx].cpu().numpy()
    S = st["S"][idx].cpu().numpy().astype(np.float64)
    A = st["A"][idx].cpu().numpy()
    W, b = st["W"], st["b"]
    scale = np.abs(f.astype(np.float64)) @ np.abs(W.astype(np.float64)).T + \
        np.abs(b.astype(np.float64))[None, :]
    acc = {"sample_crops": int(len(idx)),
           "features_bitexact": bool(np.array_equal(hist.view(np.uint32), f.view(np.uint32))),
           "max_score_err_over_condition_scale": float((np.abs(S - s64) / scale).max()),
           "max_abs_score_err_vs_fp64": float(np.abs(S - s64).max()),
           "score_tolerance": 1e-5,
           "argmax_agreement": float((A == am).mean())}
    out["accuracy"] = acc
    if "S3" in st and "split_f16_scoring" in out:
        S3 = st["S3"][idx].cpu().numpy().astype(np.float64)
        A3 = st["A3"][idx].cpu().numpy()
        out["split_f16_scoring"]["accuracy"] = {
            "sample_crops": int(len(idx)),
            "max_score_err_over_condition_scale": float((np.abs(S3 - s64) / scale).max()),
            "max_abs_score_err_vs_fp64": float(np.abs(S3 - s64).max()),
            "score_tolerance": 1e-5, "argmax_agreement": float((A3 == am).mean())}
    if latency is not None and latency.get("_fused_results"):
        out["latency"]["fused_bf16"].update(_serving_accuracy(oracle, latency, threads))
    return {"value": rn, "unit": "crops/s", "cores": threads, "kind": "oracle",
            "sample": f"ragged crops {int(idx[0])}..{int(idx[-1])} ({len(idx)} crops), features + "
                      f"FP64 scores vs {RAGGED_IDENT} identities + argmax, repeated: {cn} crops "
                      f"in {tn:.1f} s",
            "single_thread": {"value": r1, "unit": "crops/s", "cores": 1,
                              "sample": f"{c1} crops in {t1:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "threads_note": f"all-thread mode uses {threads} threads, the host CPU share of one "
                            "GPU"}


def _serving_accuracy(oracle, latency, threads, max_crops=2048):
    """BF16 serving scores against the oracle's FP64 scores of the same
    features (the served features are bit-exact FP32, checked in the tests)."""
    res = latency["_fused_results"]
    W, b = latency["_weights"]
    feats, scores, arg = [], [], []
    n = 0
    for r in res:
        if r.features is None or n >= max_crops:
            continue
        feats.append(r.features)
        scores.append(r.scores)
        arg.append(r.argmax)
        n += len(r.features)
    if not feats:
        return {}
    F = np.concatenate(feats)
    S = np.concatenate(scores).astype(np.float64)
    A = np.concatenate(arg)
    s64, am = oracle.score_f64(F, W, b, want_scores=True, n_threads=threads)
    return {"accuracy_sample_crops": int(len(F)),
            "max_abs_score_err_vs_fp64": float(np.abs(S - s64).max()),
            "argmax_agreement_vs_fp64": float((A == am).mean())}


def bench_resize(args):
    """Sec. 3's resize: every face box of 640x480 Kinect-shaped frames (1-8
    faces, sides 48-256) sampled to 200 x 200 through its frame (nearest
    sample), then features and FP32 scores against 1024 identities. One
    warped-features call (sampling kernel + feature kernel) + scoring per
    step; all frames resident in HBM."""
    import torch

    from paper_1504_01883_amd import lbpf, synth
    torch.cuda.set_device(0)
    nf, K, OUT = args.resize_frames, 1024, 200
    t0 = time.time()
    frames = [synth.make_frame(i % 16, i // 16, K) for i in range(nf)]
    print(f"[bench] generated {nf} frames in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ctx = lbpf.Context()
    D = ctx.dim
    planes = [lbpf.to_device_planes(g, z) for (g, z, _, _) in frames]
    boxes = []
    src_px = 0
    for i, (_, _, bx, _) in enumerate(frames):
        for (x, y, w, h) in bx:
            fr = lbpf.resize_frame(int(x), int(y), int(w), int(h), OUT, OUT)
            boxes.append((i, OUT, OUT, fr, fr))
            src_px += int(w) * int(h)
    n = len(boxes)
    table = lbpf.WarpBoxTable(boxes)  # marshalled once, as a serving loop would per frame set
    images = lbpf.ImageTable(planes)
    ws = torch.empty(table.workspace_bytes, dtype=torch.uint8, device="cuda")
    W, b = synth.synthetic_weights(K, D, synth.W_SERVING)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda())
    hist = torch.empty((n, D), dtype=torch.float32, device="cuda")
    S = torch.empty((n, K), dtype=torch.float32, device="cuda")
    A = torch.empty((n,), dtype=torch.int32, device="cuda")

    def step():
        ctx.features_warped(images, table, out=hist, workspace=ws)
        ctx.score(hist, wts, scores_out=S, argmax_out=A)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e = _events(4)
    fe = 0.0
    e[0].record()
    for _ in range(args.steps):
        step()
    e[1].record()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1]) / args.steps
    e[2].record()
    for _ in range(args.steps):
        ctx.features_warped(images, table, out=hist, workspace=ws)
    e[3].record()
    torch.cuda.synchronize()
    fe = e[2].elapsed_time(e[3]) / args.steps
    # Algorithmic bytes of a fused resize + features: the samples read (3 B
    # each) and the feature rows written; the staged crop's round trip is
    # what this two-kernel design adds on top.
    alg = float(n * OUT * OUT * 3 + n * D * 4)
    gbs = alg / (fe * 1e-3) / 1e9
    out = {"metric": "face crops/s (resize to 200x200 + LBP+hist+SVM)", "value": n / (ms * 1e-3),
           "unit": "crops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"resize: {n} face boxes from {nf} 640x480 frames resized to "
                                  f"{OUT}x{OUT} (nearest sample), {K} identities, FP32 scoring",
                      "crops": n, "identities": K, "dim": D, "source_pixels": src_px},
           "warped_features": {"ms": fe, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                               "algorithmic_bytes": alg,
                               "staged_bytes": float(n * OUT * OUT * 3 * 2)}}
    print(json.dumps(out), flush=True)
    wts.close()
    ctx.close()


def bench_train(args):
    """On-device one-vs-rest SVM training (Sec. 2.5) on the uniform workload's
    training set: 256 identities x 20 crops of 128x128 (5120 samples, D =
    7552), C = 1, eps = 1e-6, at most 200 epochs, dual coordinate descent.
    The timed solver is the FP32 Gram-matrix one (Gram matrix on the FP32
    matrix cores included); the FP64 device solver is timed beside it.
    Features come from the library's feature path (bit-exact with the
    oracle's, as the parity tests check). The CPU leg times the oracle trainer
    on a sample of the classes and compares its weights with the device's
    for those classes."""
    import torch

    from paper_1504_01883_amd import lbpf, synth
    torch.cuda.set_device(0)
    K, per = args.train_identities, args.train_per_identity
    t0 = time.time()
    g, z, lab = synth.make_training_set(K, per, SIDE, SIDE, synth.W_UNIFORM)
    n = len(lab)
    threads = min(CPU_SHARE, os.cpu_count() or 1)
    ctx = lbpf.Context()
    dg, dz = lbpf.to_device_planes(g.reshape(n * SIDE, SIDE), z.reshape(n * SIDE, SIDE))
    Xd, _ = ctx.features([(dg, dz)], synth.stacked_boxes(n, SIDE, SIDE))
    torch.cuda.synchronize()
    X = Xd.cpu().numpy()
    del dg, dz
    print(f"[bench] training set {n} x {X.shape[1]} in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    ld = torch.from_numpy(lab).cuda()
    for solver in ("gram", "f64"):  # warm-up: module load, first launches
        ctx.train(Xd, ld, K, max_epochs=1, solver=solver)
    torch.cuda.synchronize()
    e = _events(4)
    e[0].record()
    out_gpu = ctx.train(Xd, ld, K)
    e[1].record()
    out_f64 = ctx.train(Xd, ld, K, want_f64=True, solver="f64")
    e[2].record()
    torch.cuda.synchronize()
    gpu_s = e[0].elapsed_time(e[1]) * 1e-3
    f64_s = e[1].elapsed_time(e[2]) * 1e-3
    epochs = out_gpu["epochs"].cpu().numpy()
    W32 = out_gpu["W"].cpu().numpy().astype(np.float64)
    W64 = out_f64["W64"].cpu().numpy()
    # CPU leg: the oracle on a sample of classes, relabelled so the sampled
    # classes are 0..m-1.
    import oracle
    m = min(K, 2 * threads)
    lab_s = np.where(lab < m, lab, m).astype(np.int32)  # everything else is "rest"
    t0 = time.perf_counter()
    W_ref, _, ep_ref = oracle.train_ovr_f64(X, lab_s, m, n_threads=threads)
    cpu_s = time.perf_counter() - t0
    scale = max(np.abs(W_ref).max(), 1e-30)
    err = float(np.abs(W32[:m] - W_ref).max() / scale)
    err64 = float(np.abs(W64[:m] - W_ref).max() / scale)
    res = {"metric": "SVM training: identities trained per second", "value": K / gpu_s,
           "unit": "identities/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"one-vs-rest training: {K} identities x {per} crops 128x128 "
                                  f"({n} samples, D = {X.shape[1]}), C = 1, eps = 1e-6, <= 200 "
                                  "epochs", "samples": n, "identities": K, "dim": int(X.shape[1])},
           "gpu_seconds": gpu_s, "epochs_max": int(epochs.max()),
           "epochs_mean": float(epochs.mean()),
           "cpu_baseline": {"value": m / cpu_s, "unit": "identities/s", "cores": threads,
                            "kind": "oracle", "sample": f"{m} of the {K} identities, "
                                                        f"{cpu_s:.1f} s"},
           "max_rel_weight_diff_vs_oracle": err, "oracle_epochs_sample": int(ep_ref),
           "solver": "FP32 Gram matrix (matrix-core GEMM) + dual coordinate descent",
           "f64_solver": {"value": K / f64_s, "seconds": f64_s,
                          "max_rel_weight_diff_vs_oracle": err64,
                          "epochs_max": int(out_f64["epochs"].cpu().numpy().max())}}
    print(json.dumps(res), flush=True)
    ctx.close()


PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0, "f16x3": 2500.0}
# Matrix-core flops executed per algorithmic flop: the split FP16 mode runs
# three FP16 products.
EXEC_FACTOR = {"fp32": 1, "bf16": 1, "fp16": 1, "fp8": 1, "f16x3": 3}
LP_CHUNK = 16384  # feature rows the library quantises per pass


def bench_precision(args):
    """Precision: N x 7552 features scored against K identities with FP32,
    BF16, FP16 and FP8-e4m3 operands (FP32 accumulation). The feature rows are
    distinct: the features of 8192 uniform-generator crops, block j of 8192
    rows cyclically shifted by j whole 59-bin cells (the GEMM's time does not
    depend on the values). The CPU leg scores sampled rows of every
    16,384-row chunk with the FP64 oracle: that is both the CPU baseline and
    the reference of the stated errors and argmax agreement."""
    import torch

    from paper_1504_01883_amd import lbpf, synth
    torch.cuda.set_device(0)
    N, K = args.precision_rows, args.precision_identities
    distinct = min(8192, N)
    g, z, _ = synth.make_crops(distinct, SIDE, SIDE, synth.W_PRECISION, N_IDENT)
    ctx = lbpf.Context()
    D = ctx.dim
    dg, dz = lbpf.to_device_planes(g.reshape(-1, SIDE), z.reshape(-1, SIDE))
    base, _ = ctx.features([(dg, dz)], synth.stacked_boxes(distinct, SIDE, SIDE))
    X = torch.cat([torch.roll(base, shifts=59 * j, dims=1)
                   for j in range((N + distinct - 1) // distinct)])[:N].contiguous()
    del base, dg, dz
    W, b = synth.synthetic_weights(K, D, synth.W_PRECISION)
    Wd, bd = torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()
    S = torch.empty((N, K), dtype=torch.float32, device="cuda")
    A = torch.empty((N,), dtype=torch.int32, device="cuda")
    # Sampled rows: the first and last row of every chunk and 62 more per chunk.
    rng = np.random.default_rng(7)
    sample = []
    for c0 in range(0, N, LP_CHUNK):
        c1 = min(N, c0 + LP_CHUNK)
        sample += [c0, c1 - 1] + list(rng.integers(c0, c1, min(62, c1 - c0)))
    sample = np.unique(np.array(sample, np.int64))
    flops = 2.0 * N * K * D
    res, got = {}, {}
    for prec in ("fp32", "bf16", "fp16", "fp8", "f16x3"):
        wts = ctx.weights(Wd, bd, precision=prec)
        steps = max(1, min(args.steps, 3 if prec == "fp32" else 10))
        ctx.score(X, wts, scores_out=S, argmax_out=A)
        torch.cuda.synchronize()
        e = _events(2)
        e[0].record()
        for _ in range(steps):
            ctx.score(X, wts, scores_out=S, argmax_out=A)
        e[1].record()
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1]) / steps
        tf = flops / (ms * 1e-3) / 1e12
        idx = torch.from_numpy(sample).cuda()
        got[prec] = (S[idx].double().cpu().numpy(), A[idx].cpu().numpy())
        # The same call asking for the argmax only (no score matrix written).
        A2 = torch.empty_like(A)
        ctx.score(X, wts, want_scores=False, argmax_out=A2)
        torch.cuda.synchronize()
        same = bool(torch.equal(A2, A))
        e[0].record()
        for _ in range(steps):
            ctx.score(X, wts, want_scores=False, argmax_out=A2)
        e[1].record()
        torch.cuda.synchronize()
        ms_a = e[0].elapsed_time(e[1]) / steps
        tf_a = flops / (ms_a * 1e-3) / 1e12
        xf = EXEC_FACTOR[prec]
        res[prec] = {"ms": ms, "tflops": tf, "peak_tflops": PEAKS_TFLOPS[prec],
                     "mfma_frac": xf * tf / PEAKS_TFLOPS[prec],
                     "includes": "feature-row quantisation + GEMM + argmax" if prec != "fp32"
                                 else "GEMM + argmax",
                     "argmax_only": {"ms": ms_a, "tflops": tf_a,
                                     "mfma_frac": xf * tf_a / PEAKS_TFLOPS[prec],
                                     "argmax_equal_to_with_scores": same}}
        if xf != 1:
            res[prec]["note"] = (f"tflops counts the product's 2 N K D flops; the matrix cores "
                                 f"execute {xf}x that in FP16 (mfma_frac)")
        print(f"[bench] {prec}: {ms:.2f} ms, {tf:.1f} TFLOP/s; argmax only {ms_a:.2f} ms",
              file=sys.stderr, flush=True)
        wts.close()
    Xs = X[torch.from_numpy(sample).cuda()].cpu().numpy()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = min(CPU_SHARE, os.cpu_count() or 1)
        t0 = time.perf_counter()
        S64, A64 = oracle.score_f64(Xs, W, b, want_scores=True, n_threads=threads)
        dt = time.perf_counter() - t0
        cond = np.abs(Xs.astype(np.float64)) @ np.abs(W.astype(np.float64)).T + \
            np.abs(b.astype(np.float64))[None, :]
        for prec in res:
            Sg, Ag = got[prec]
            res[prec]["max_abs_err_vs_fp64"] = float(np.abs(Sg - S64).max())
            res[prec]["max_err_over_condition_scale"] = float((np.abs(Sg - S64) / cond).max())
            res[prec]["argmax_agreement_vs_fp64"] = float((Ag == A64).mean())
        cpu = {"value": 2.0 * len(sample) * K * D / dt / 1e12, "unit": "TFLOP/s (FP64)",
               "cores": threads, "kind": "oracle",
               "sample": f"{len(sample)} rows from every {LP_CHUNK}-row chunk scored against "
                         f"{K} identities in {dt:.1f} s"}
    best = max(res, key=lambda k: res[k]["tflops"])
    out = {"metric": "scoring TFLOP/s by operand precision", "value": res[best]["tflops"],
           "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"precision: {N} x {D} features vs {K} identities",
                      "rows": N, "identities": K, "dim": D, "flops_per_launch": flops,
                      "error_sample_rows": int(len(sample))},
           "by_precision": res, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
