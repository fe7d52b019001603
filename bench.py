#!/usr/bin/env python3
"""Benchmark of the non-separable 2-D CDF 5/3 DWT on one MI355X.

Timed step: on one resident 8192 x 8192 float32 image (6 levels), the whole
hot path once: forward transform, inverse transform, and adjoint (W^T g) of a
coefficient-shaped gradient.  Inputs are generated on the device before the
timed region; two buffer sets alternate between steps so that the 256 MB
Infinity Cache cannot hold a step's input from the previous step.  Nothing
else is recorded inside the timed steps.  Before the warmup, dwt2_tune picks
the work-item heights of each direction's launches for this shape (a
one-off of some tens of milliseconds, outside the timed region; every other
workload below is tuned the same way before it is timed).

value = pixels transformed per second over the step, in Gpixel/s (each of the
three passes counts the image's 8192^2 pixels once, whatever the number of
levels).

roofline: right after the timed steps, the same steps run again with the
library's timing probe (dwt2_set_probe) recording HIP events on the call's
stream around one launch at a time, for every launch of every direction
(dwt2_launch_levels lists them).  The dominant kernel is the launch with the
longest mean duration; achieved = the algorithmic bytes of the levels it
computes (each level reads its input once and writes as many coefficients)
/ that mean duration.  Every launch's figure is in detail.launches.

cpu_baseline: the CPU oracle (float64 numpy, untuned) on the host, before the
GPU is touched: the step's three passes on a 4096 x 4096 image of the same
generator, 6 levels -- once per core in parallel worker processes (the
figure reported) and alone on one thread (median of several runs).

Side measurements in "detail": per-direction times and fractions, the
separable lifting baselines (per-step passes and LDS-tiled) against the
non-separable forward (the paper's comparison), the CDF 9/7 forward/inverse
(strip kernels) and its four-step tiled forward against the eight-step one on
the same tiles,
the other workloads of the transform (512^2 one level; 16384^2 int32 six
levels; the ragged 256-image batch, batched vs plain; 32 x 3 x 1024^2 four
levels, forward and adjoint alone and through autograd), one GPU's strip of a
split 16384^2 image, and a device copy ceiling.

--sweep prints, instead, the two comparisons of the paper's §4 redone on this
GPU: the forward's time against the image edge (512 .. 16384, 6 levels) for
the product path, the LDS-tiled non-separable (two barrier steps), adapted
(two, fewer operations) and separable (four) kernels and the separable-pass
baseline, and the CDF 9/7 (its strip kernels, and its tiled kernel with four
steps against the separable counterpart on the same tiles with eight); and
the level-1 time of 8192^2 against the work-item
shape (segment height x prefetch chunk), the counterpart of the paper's
tile-size experiment.

--only PART runs one part untimed, for profiling (rocprofv3).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sweep] [--only PART]
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
METRIC = "Gpixel/s and % HBM roofline, 2-D CDF 5/3 fwd/adjoint; batched vs plain"
HBM_PEAK_GBPS = 8000.0


def level_sizes(w, h, levels):
    out = [(w, h)]
    for _ in range(levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        out.append((w, h))
    return out


def alg_bytes(w, h, levels, elem=4):
    """Each level reads its input region once and writes as many coefficients."""
    return sum(2 * elem * a * b for (a, b) in level_sizes(w, h, levels)[:-1])


def kernel_sources_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1708_07853_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key):
    """HBM bytes per launch of one kernel from the committed rocprofv3 counter
    summaries (profiles/*_traffic.txt), if they were taken on the current
    kernel sources; None otherwise."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith("_traffic.txt"):
            continue
        rec = {}
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if line.startswith("#") or ":" not in line:
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                rec[k] = v
        if rec.get("kernel_sources_sha256_16") != kernel_sources_digest():
            continue
        v = rec.get(f"{kernel_key}_bytes_per_launch")
        if v:
            return float(v)
    return None


class Timer:
    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, reps):
        t = self.torch
        ev = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        t.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]



def _cpu_step(w, h, levels, seed, barrier=None):
    """One step of the oracle (forward, inverse, adjoint) on one image of the
    generator; returns (start, end) of the oracle's work on the monotonic
    clock.  With a barrier, the image is built first and the timing starts
    once every worker is ready."""
    import oracle
    from paper_1708_07853_amd import synth
    x = synth.image(w, h, seed).astype(np.float64)
    g = np.random.default_rng(seed + 1).normal(size=x.shape) * 16
    if barrier is not None:
        barrier.wait()
    t = time.perf_counter()
    c = oracle.fwd(x, levels)
    oracle.inv(c, levels)
    oracle.adj(g, levels)
    return t, time.perf_counter()


def _cpu_worker(q, barrier, w, h, levels, seed):
    q.put(_cpu_step(w, h, levels, seed, barrier))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w=4096, h=4096, levels=6, runs=3):
    """The oracle on the host's cores (see the module doc).  Runs before any
    GPU work; the parallel workers are forked processes."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, 16))
    single = []
    for _ in range(runs):
        t0, t1 = _cpu_step(w, h, levels, 2)
        single.append(t1 - t0)
    t_single = float(np.median(single))
    ctx = mp.get_context("fork")
    q, barrier = ctx.Queue(), ctx.Barrier(workers)
    procs = [ctx.Process(target=_cpu_worker, args=(q, barrier, w, h, levels, 2 + k)) for k in range(workers)]
    for p in procs:
        p.start()
    spans = [q.get() for _ in procs]
    for p in procs:
        p.join()
    t_all = max(e for _, e in spans) - min(b for b, _ in spans)
    px = 3 * w * h                     # three passes per step
    return {
        "value": round(workers * px / t_all / 1e9, 5), "unit": "Gpixel/s", "cores": workers, "kind": "oracle",
        "sample": (f"one step (float64 forward + inverse + adjoint, {levels} levels) of a {w}x{h} image of the "
                   f"same generator per worker process, {workers} processes in parallel, {t_all:.2f} s from the "
                   f"first start to the last end; the benchmark's 8192x8192 image has 4x the pixels"),
        "ns_per_pel": round(t_all / (workers * px) * 1e9, 3),
        "single_thread": {"Gpx_s": round(px / t_single / 1e9, 5), "ns_per_pel": round(t_single / px * 1e9, 2),
                          "median_s": round(t_single, 3), "runs": runs},
        "host": {"model": _cpu_model(), "cpu_count": os.cpu_count(), "affinity": avail},
    }


def _tiled97(f):
    """Run f with the CDF 9/7 on its LDS-tiled kernels at every level (the same
    tiles as the separable 9/7 comparison kernel) instead of the default
    choice, which takes the strip kernels for most levels."""
    os.environ["DWT2_CDF97_TILED"] = "1"
    try:
        return f()
    finally:
        os.environ.pop("DWT2_CDF97_TILED", None)


def tune_passes(dwt, passes, levels):
    """dwt2_tune for each (direction, input, output, workspace) of a workload."""
    for d, x, out, ws in passes:
        dwt.tune(d, x, levels, out=out, workspace=ws)


def _med(x):
    return float(np.median(x))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-detail", action="store_true", help="skip the side measurements")
    ap.add_argument("--only", choices=["step", "fwd", "fwd1", "inv", "bwd", "copy", "fwd97", "inv97", "c1", "int16k",
                                       "ragged", "c5"], default=None,
                    help="profiling aid: run only this part, untimed (fwd1: the level-1 forward alone as a "
                         "1-level call; c1: 512^2, 1 level; int16k: 16384^2 int32 forward + inverse; ragged: the "
                         "256-image batch, batched forward; c5: 32x3x1024^2 forward + adjoint)")
    ap.add_argument("--sweep", action="store_true",
                    help="print the edge-size and work-item-shape sweeps instead of the benchmark line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not (args.no_cpu_baseline or args.only or args.sweep):
        cpu = cpu_baseline()           # before the GPU is touched

    import torch
    import paper_1708_07853_amd as dwt
    from paper_1708_07853_amd import synth, _lib

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    timer = Timer(torch)

    if args.sweep:
        sweep(torch, dwt, synth, dev, timer)
        return
    if args.only in ("c1", "int16k", "ragged", "c5"):
        only_workload(args.only, max(1, args.steps), torch, dwt, synth, dev)
        return

    W = H = 8192
    L = 6
    npx = W * H
    sets = []
    for s in range(2):
        x = synth.image_device(W, H, 2 + 100 * s, device=dev)
        g = torch.randn((H, W), generator=torch.Generator(device=dev).manual_seed(6 + s), device=dev) * 16
        sets.append(dict(x=x, c=torch.empty_like(x), r=torch.empty_like(x), g=g, gx=torch.empty_like(x)))
    wsb = dwt.workspace_size(W, H, L)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

    def fwd(s):
        dwt.fwd(s["x"], L, out=s["c"], workspace=ws)

    def inv(s):
        dwt.inv(s["c"], L, out=s["r"], workspace=ws)

    def bwd(s):
        dwt.bwd(s["g"], L, out=s["gx"], workspace=ws)

    passes = {"fwd": fwd, "inv": inv, "bwd": bwd}
    s0 = sets[0]
    fwd(s0)  # the inverse's tuning input
    tune_passes(dwt, [("fwd", s0["x"], s0["c"], ws), ("inv", s0["c"], s0["r"], ws), ("bwd", s0["g"], s0["gx"], ws)], L)

    if args.only in ("fwd97", "inv97"):
        dwt.fwd_cdf97(s0["x"], L, out=s0["c"], workspace=ws)
        tune_passes(dwt, [("fwd_cdf97", s0["x"], s0["c"], ws), ("inv_cdf97", s0["c"], s0["r"], ws)], L)
    if args.only:
        reps = max(1, args.steps)
        for i in range(reps):
            s = sets[i & 1]
            if args.only in ("step", "fwd"):
                fwd(s)
            if args.only == "fwd1":
                dwt.fwd(s["x"], 1, out=s["c"], workspace=ws)
            if args.only in ("step", "inv"):
                inv(s)
            if args.only in ("step", "bwd"):
                bwd(s)
            if args.only == "copy":
                s["c"].copy_(s["x"])
            if args.only == "fwd97":
                dwt.fwd_cdf97(s["x"], L, out=s["c"], workspace=ws)
            if args.only == "inv97":
                dwt.inv_cdf97(s["c"], L, out=s["r"], workspace=ws)
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "reps": reps}))
        return

    # ---- warmup + timed steps (nothing but the three passes) ---------------
    for i in range(args.warmup):
        s = sets[i & 1]
        fwd(s); inv(s); bwd(s)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for e in ev:  # create the HIP events before the timed region
        for x_ in e:
            x_.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s = sets[i & 1]
        e = ev[i]
        e[0].record(); fwd(s); e[1].record(); inv(s); e[2].record(); bwd(s); e[3].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    per_dir = {k: _med([e[j].elapsed_time(e[j + 1]) for e in ev]) for j, k in enumerate(("fwd", "inv", "bwd"))}
    value = 3 * npx / (ms_step * 1e-3) / 1e9

    # ---- every launch of the step, probed one at a time, same steps again ---
    sizes = level_sizes(W, H, L)
    launches = []
    reps = max(10, min(args.steps, 20))
    for dname in ("fwd", "inv", "bwd"):
        for (first, last) in dwt.launch_levels(W, H, L, dname):
            pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for i, (b, e_) in enumerate(pe):
                s = sets[i & 1]
                dwt.set_probe(dname, first, b, e_)
                fwd(s); inv(s); bwd(s)
            torch.cuda.synchronize()
            dwt.set_probe(None)
            t = [b.elapsed_time(e_) for b, e_ in pe]
            nbytes = sum(2 * 4 * a * b_ for (a, b_) in sizes[first - 1:last])
            launches.append({"dir": dname, "levels": [first, last], "mean_ms": round(float(np.mean(t)), 5),
                             "p10_p90_ms": [round(float(np.percentile(t, 10)), 5),
                                            round(float(np.percentile(t, 90)), 5)],
                             "alg_bytes": nbytes,
                             "frac_of_8TBps": round(nbytes / (float(np.mean(t)) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)})
    dom = max(launches, key=lambda r: r["mean_ms"])
    achieved = dom["alg_bytes"] / (dom["mean_ms"] * 1e-3) / 1e9
    lv = dom["levels"]
    kname = f"{dom['dir']} launch of levels {lv[0]}..{lv[1]} of the 8192x8192 6-level transform"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": read_traffic(f"{dom['dir']}_levels_{lv[0]}_{lv[1]}_8192"),
                "kernel": kname, "bytes_per_launch": dom["alg_bytes"], "avg_launch_ms": dom["mean_ms"],
                "launch_ms_p10_p90": dom["p10_p90_ms"], "launches_probed": reps}

    alg = alg_bytes(W, H, L)
    detail = {"ms_per_direction": {k: round(v, 4) for k, v in per_dir.items()},
              "direction_GBps_alg": {k: round(alg / (v * 1e-3) / 1e9, 1) for k, v in per_dir.items()},
              "direction_frac_of_8TBps": {k: round(alg / (v * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
                                          for k, v in per_dir.items()},
              "alg_bytes_per_direction": alg, "launches": launches}

    if not args.no_detail:
        side_measurements(detail, sets, ws, fwd, W, H, L, npx, torch, dwt, synth, dev, timer)

    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "8192x8192 float32 image, 6 levels: forward + inverse + adjoint per step "
                                  "(non-separable CDF 5/3, symmetric extension)",
                      "width": W, "height": H, "levels": L, "parallelism": "none (1 GPU)"},
           "roofline": roofline, "cpu_baseline": cpu, "detail": detail}
    print(json.dumps(out))


def only_workload(part, reps, torch, dwt, synth, dev):
    """One of the other workloads, untimed, for profiling."""
    if part == "c1":
        x = synth.image_device(512, 512, 1, device=dev)
        c = torch.empty_like(x)
        ws = torch.empty(max(1, dwt.workspace_size(512, 512, 1)), dtype=torch.uint8, device=dev)
        tune_passes(dwt, [("fwd", x, c, ws)], 1)
        for _ in range(reps):
            dwt.fwd(x, 1, out=c, workspace=ws)
    elif part == "int16k":
        xi = synth.image_device(16384, 16384, 3, dtype=torch.int32, device=dev)
        ci, ri = torch.empty_like(xi), torch.empty_like(xi)
        wsi = torch.empty(dwt.workspace_size(16384, 16384, 6, mode=1), dtype=torch.uint8, device=dev)
        dwt.fwd(xi, 6, out=ci, workspace=wsi)
        tune_passes(dwt, [("fwd", xi, ci, wsi), ("inv", ci, ri, wsi)], 6)
        for _ in range(reps):
            dwt.fwd(xi, 6, out=ci, workspace=wsi)
            dwt.inv(ci, 6, out=ri, workspace=wsi)
    elif part == "ragged":
        sizes = synth.ragged_sizes(256, 4)
        imgs = [synth.image_device(w, h, 4000 + i, device=dev) for i, (w, h) in enumerate(sizes)]
        outs = [torch.empty_like(t) for t in imgs]
        bws = torch.empty(dwt.batched_workspace_size(imgs, 3), dtype=torch.uint8, device=dev)
        for _ in range(reps):
            dwt.fwd_batched(imgs, 3, outs=outs, workspace=bws)
    elif part == "c5":
        xb = torch.stack([synth.image_device(1024, 1024, 5000 + k, device=dev) for k in range(96)])
        xb = xb.reshape(32, 3, 1024, 1024)
        c, gx = torch.empty_like(xb), torch.empty_like(xb)
        ws = torch.empty(dwt.workspace_size(1024, 1024, 4, batch=96), dtype=torch.uint8, device=dev)
        dwt.fwd(xb, 4, out=c, workspace=ws)
        tune_passes(dwt, [("fwd", xb, c, ws), ("bwd", c, gx, ws)], 4)
        for _ in range(reps):
            dwt.fwd(xb, 4, out=c, workspace=ws)
            dwt.bwd(c, 4, out=gx, workspace=ws)
    torch.cuda.synchronize()
    print(json.dumps({"only": part, "reps": reps}))


def side_measurements(detail, sets, ws, fwd, W, H, L, npx, torch, dwt, synth, dev, timer):
    k = [0]
    # the paper's comparison: separable lifting (eq. (3), one pass per
    # step) against the fused non-separable scheme, same image, 6 levels
    wss = torch.empty(dwt.separable_workspace_size(W, H, L), dtype=torch.uint8, device=dev)

    def sep_fwd():
        k[0] ^= 1
        s_ = sets[k[0]]
        dwt.fwd_separable(s_["x"], L, out=s_["c"], workspace=wss)

    def fused_fwd():
        k[0] ^= 1
        fwd(sets[k[0]])

    def lds_fwd(scheme):
        def f():
            k[0] ^= 1
            s_ = sets[k[0]]
            dwt.fwd_lds(s_["x"], L, scheme, out=s_["c"], workspace=ws)
        return f

    for _ in range(3):
        sep_fwd()
    ts = _med(timer(sep_fwd, 20))
    tf = _med(timer(fused_fwd, 20))
    lds = {}
    for scheme in ("separable", "nonseparable", "adapted"):
        f = lds_fwd(scheme)
        for _ in range(3):
            f()
        lds[scheme] = _med(timer(f, 20))
    detail["separable_vs_nonseparable_fwd_8192_L6"] = {
        "separable_ms": round(ts, 4), "nonseparable_ms": round(tf, 4),
        "speedup": round(ts / tf, 3),
        "separable_hbm_passes_per_level": 4, "nonseparable_hbm_passes_per_level": 1,
        "lds_tiled_separable_ms": round(lds["separable"], 4),
        "lds_tiled_nonseparable_ms": round(lds["nonseparable"], 4),
        "lds_tiled_adapted_ms": round(lds["adapted"], 4),
        "lds_tiled_speedup_of_two_steps_over_four": round(lds["separable"] / lds["nonseparable"], 3)}
    del wss
    # CDF 9/7 (float32), the same image and levels: forward and inverse
    s0 = sets[0]
    dwt.fwd_cdf97(s0["x"], L, out=s0["c"], workspace=ws)  # the inverse's tuning input
    tune_passes(dwt, [("fwd_cdf97", s0["x"], s0["c"], ws), ("inv_cdf97", s0["c"], s0["r"], ws)], L)
    t97 = {}
    for name, f in (("fwd", lambda s_: dwt.fwd_cdf97(s_["x"], L, out=s_["c"], workspace=ws)),
                    ("inv", lambda s_: dwt.inv_cdf97(s_["c"], L, out=s_["r"], workspace=ws)),
                    ("fwd_tiled", lambda s_: _tiled97(lambda: dwt.fwd_cdf97(s_["x"], L, out=s_["r"], workspace=ws))),
                    ("fwd_sep", lambda s_: dwt.fwd_cdf97_separable(s_["x"], L, out=s_["r"], workspace=ws))):
        def g(f=f):
            k[0] ^= 1
            f(sets[k[0]])
        for _ in range(3):
            g()
        t97[name] = _med(timer(g, 20))
    rt = float((dwt.inv_cdf97(dwt.fwd_cdf97(sets[0]["x"], L), L) - sets[0]["x"]).abs().max())
    detail["cdf97_8192_L6"] = {
        "fwd_ms": round(t97["fwd"], 4), "inv_ms": round(t97["inv"], 4),
        "fwd_tiled_4_steps_ms": round(t97["fwd_tiled"], 4),
        "fwd_separable_8_steps_ms": round(t97["fwd_sep"], 4),
        "speedup_of_4_steps_over_8_same_tiles": round(t97["fwd_sep"] / t97["fwd_tiled"], 3),
        "fwd_Gpx_s": round(npx / (t97["fwd"] * 1e-3) / 1e9, 1),
        "inv_Gpx_s": round(npx / (t97["inv"] * 1e-3) / 1e9, 1),
        "fwd_frac_of_8TBps": round(alg_bytes(W, H, L) / (t97["fwd"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "inv_frac_of_8TBps": round(alg_bytes(W, H, L) / (t97["inv"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "roundtrip_max_abs_err": rt}
    # 512^2 float32, one level (launch-bound; two buffer sets alternate)
    xs1 = [synth.image_device(512, 512, 1 + 100 * s_, device=dev) for s_ in range(2)]
    cs1 = [torch.empty_like(x_) for x_ in xs1]
    ws1 = torch.empty(max(1, dwt.workspace_size(512, 512, 1)), dtype=torch.uint8, device=dev)
    tune_passes(dwt, [("fwd", xs1[0], cs1[0], ws1)], 1)

    def c1(i=[0]):
        i[0] ^= 1
        dwt.fwd(xs1[i[0]], 1, out=cs1[i[0]], workspace=ws1)
    for _ in range(10):
        c1()
    t1 = timer(c1, 100)
    detail["config1_512_L1_fwd"] = {"us_median": round(_med(t1) * 1e3, 2),
                                    "us_p10_p90": [round(float(np.percentile(t1, 10)) * 1e3, 2),
                                                   round(float(np.percentile(t1, 90)) * 1e3, 2)],
                                    "Gpx_s": round(512 * 512 / (_med(t1) * 1e-3) / 1e9, 2)}
    del xs1, cs1, ws1
    # one GPU's share of a 16384^2 image split into 8 horizontal strips:
    # 2048 rows plus the one-quadruple (2-row) halo the fused level
    # needs from each neighbour, level 1 forward
    xs_ = [synth.image_device(16384, 2048 + 4, 7 + s_, device=dev) for s_ in range(2)]
    cs_ = [torch.empty_like(x_) for x_ in xs_]
    wsx = torch.empty(max(1, dwt.workspace_size(16384, 2052, 1)), dtype=torch.uint8, device=dev)
    tune_passes(dwt, [("fwd", xs_[0], cs_[0], wsx)], 1)

    def strip(i=[0]):
        i[0] ^= 1
        dwt.fwd(xs_[i[0]], 1, out=cs_[i[0]], workspace=wsx)
    for _ in range(3):
        strip()
    tsx = _med(timer(strip, 20))
    detail["strip_share_16384x2052_L1"] = {
        "ms": round(tsx, 4), "GBps_alg": round(2 * 4 * 16384 * 2052 / (tsx * 1e-3) / 1e9, 1),
        "frac_of_8TBps": round(2 * 4 * 16384 * 2052 / (tsx * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    del xs_, cs_, wsx
    # copy ceiling: read + write of 1 GiB
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    cp = timer(lambda: b.copy_(a), 20)
    detail["copy_ceiling_GBps"] = round(2 * a.numel() * 4 / (_med(cp) * 1e-3) / 1e9, 1)
    del a, b
    # integer 16384^2, 6 levels, forward + inverse
    xi = synth.image_device(16384, 16384, 3, dtype=torch.int32, device=dev)
    ci, ri = torch.empty_like(xi), torch.empty_like(xi)
    wsi = torch.empty(dwt.workspace_size(16384, 16384, 6, mode=1), dtype=torch.uint8, device=dev)
    dwt.fwd(xi, 6, out=ci, workspace=wsi)
    tune_passes(dwt, [("fwd", xi, ci, wsi), ("inv", ci, ri, wsi)], 6)
    for _ in range(2):
        dwt.fwd(xi, 6, out=ci, workspace=wsi); dwt.inv(ci, 6, out=ri, workspace=wsi)
    tf = timer(lambda: dwt.fwd(xi, 6, out=ci, workspace=wsi), 10)
    ti = timer(lambda: dwt.inv(ci, 6, out=ri, workspace=wsi), 10)
    a16 = alg_bytes(16384, 16384, 6)
    detail["int32_16384_L6"] = {
        "fwd_ms": round(_med(tf), 4), "inv_ms": round(_med(ti), 4),
        "fwd_Gpx_s": round(16384 ** 2 / (_med(tf) * 1e-3) / 1e9, 1),
        "inv_Gpx_s": round(16384 ** 2 / (_med(ti) * 1e-3) / 1e9, 1),
        "fwd_frac_of_8TBps": round(a16 / (_med(tf) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "inv_frac_of_8TBps": round(a16 / (_med(ti) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "roundtrip_exact": bool(torch.equal(ri, xi))}
    del xi, ci, ri, wsi
    # ragged batch: 256 images, (64..4096)^2, 3 levels
    sizes = synth.ragged_sizes(256, 4)
    imgs = [synth.image_device(w, h, 4000 + i, device=dev) for i, (w, h) in enumerate(sizes)]
    outs = [torch.empty_like(t) for t in imgs]
    wss = [torch.empty(max(1, dwt.workspace_size(w, h, 3)), dtype=torch.uint8, device=dev) for (w, h) in sizes]
    bws = torch.empty(dwt.batched_workspace_size(imgs, 3), dtype=torch.uint8, device=dev)

    def plain():
        for im, o, w_ in zip(imgs, outs, wss):
            dwt.fwd(im, 3, out=o, workspace=w_)

    t_build = time.perf_counter()
    dwt.fwd_batched(imgs, 3, outs=outs, workspace=bws)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t_build
    plain()
    tp = timer(plain, 10)
    tb = timer(lambda: dwt.fwd_batched(imgs, 3, outs=outs, workspace=bws), 10)
    gpx = sum(w * h for w, h in sizes)
    detail["ragged_256_L3"] = {
        "plain_ms": round(_med(tp), 3), "batched_ms": round(_med(tb), 3),
        "plain_images_per_s": round(256 / (_med(tp) * 1e-3), 1),
        "batched_images_per_s": round(256 / (_med(tb) * 1e-3), 1),
        "batched_Gpx_s": round(gpx / (_med(tb) * 1e-3) / 1e9, 1),
        "batched_GBps_alg": round(sum(alg_bytes(w, h, 3) for w, h in sizes) / (_med(tb) * 1e-3) / 1e9, 1),
        "batched_frac_of_8TBps": round(sum(alg_bytes(w, h, 3) for w, h in sizes) / (_med(tb) * 1e-3) / 1e9
                                       / HBM_PEAK_GBPS, 4),
        "batched_over_plain": round(_med(tp) / _med(tb), 3),
        "first_call_s": round(t_build, 3), "Gpx": round(gpx / 1e9, 3)}
    # batched inverse and adjoint on the same set (coefficients from above)
    recs = [torch.empty_like(t) for t in imgs]

    def plain_inv():
        for o, r, w_ in zip(outs, recs, wss):
            dwt.inv(o, 3, out=r, workspace=w_)

    dwt.inv_batched(outs, 3, outs=recs, workspace=bws)
    dwt.bwd_batched(outs, 3, outs=recs, workspace=bws)
    plain_inv()
    tpi = timer(plain_inv, 10)
    tbi = timer(lambda: dwt.inv_batched(outs, 3, outs=recs, workspace=bws), 10)
    tbb = timer(lambda: dwt.bwd_batched(outs, 3, outs=recs, workspace=bws), 10)
    detail["ragged_256_L3"].update({
        "inv_plain_ms": round(_med(tpi), 3), "inv_batched_ms": round(_med(tbi), 3),
        "adj_batched_ms": round(_med(tbb), 3)})
    del imgs, outs, wss, bws, recs
    # 32 x 3 x 1024^2, 4 levels: the forward and the adjoint alone, then
    # forward + loss + backward through autograd
    xb = torch.stack([synth.image_device(1024, 1024, 5000 + k_, device=dev) for k_ in range(96)])
    xb = xb.reshape(32, 3, 1024, 1024)
    c5, g5 = torch.empty_like(xb), torch.empty_like(xb)
    ws5 = torch.empty(dwt.workspace_size(1024, 1024, 4, batch=96), dtype=torch.uint8, device=dev)
    dwt.fwd(xb, 4, out=c5, workspace=ws5)
    tune_passes(dwt, [("fwd", xb, c5, ws5), ("bwd", c5, g5, ws5)], 4)
    for _ in range(3):
        dwt.fwd(xb, 4, out=c5, workspace=ws5)
        dwt.bwd(c5, 4, out=g5, workspace=ws5)
    t5f = timer(lambda: dwt.fwd(xb, 4, out=c5, workspace=ws5), 20)
    t5b = timer(lambda: dwt.bwd(c5, 4, out=g5, workspace=ws5), 20)
    a5 = 96 * alg_bytes(1024, 1024, 4)
    detail["config5_32x3x1024_L4"] = {
        "fwd_ms": round(_med(t5f), 4), "bwd_ms": round(_med(t5b), 4),
        "fwd_Gpx_s": round(96 * 1024 ** 2 / (_med(t5f) * 1e-3) / 1e9, 1),
        "bwd_Gpx_s": round(96 * 1024 ** 2 / (_med(t5b) * 1e-3) / 1e9, 1),
        "fwd_frac_of_8TBps": round(a5 / (_med(t5f) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "bwd_frac_of_8TBps": round(a5 / (_med(t5b) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "alg_bytes_per_direction": a5}
    del c5, g5, ws5
    xb.requires_grad_()
    # loss: sum over levels k = 1..4 of 2^k times the L1 norms of HL_k, LH_k, HH_k
    wk = torch.zeros((1024, 1024), device=dev)
    dims = level_sizes(1024, 1024, 4)
    for k_ in range(4, 0, -1):
        (w0, h0), (w1, h1) = dims[k_ - 1], dims[k_]
        wk[:h0, :w0] = 2.0 ** k_
        wk[:h1, :w1] = 0.0

    def fb():
        y = dwt.DWT2Function.apply(xb, 4)
        (y.abs() * wk).sum().backward()

    fb()
    ta = timer(fb, 5)
    detail["config5_32x3x1024_L4"]["autograd_fwd_loss_bwd_ms"] = round(_med(ta), 3)
    del xb
    torch.cuda.empty_cache()


def sweep(torch, dwt, synth, dev, timer, reps=20):
    """The paper's §4 experiments redone on this GPU (see the module doc)."""
    def med(f):
        for _ in range(3):
            f(0)
        i = [0]

        def g():
            i[0] ^= 1
            f(i[0])
        return float(np.median(timer(g, reps)))

    for edge in (512, 1024, 2048, 4096, 8192, 16384):
        L = 6
        xs = [synth.image_device(edge, edge, 2 + 100 * s, device=dev) for s in range(2)]
        outs = [torch.empty_like(x) for x in xs]
        ws = torch.empty(dwt.separable_workspace_size(edge, edge, L), dtype=torch.uint8, device=dev)
        row = {"sweep": "edge", "edge": edge, "levels": L}
        variants = {
            "product": lambda s: dwt.fwd(xs[s], L, out=outs[s], workspace=ws),
            "lds_nonseparable": lambda s: dwt.fwd_lds(xs[s], L, "nonseparable", out=outs[s], workspace=ws),
            "lds_separable": lambda s: dwt.fwd_lds(xs[s], L, "separable", out=outs[s], workspace=ws),
            "lds_adapted": lambda s: dwt.fwd_lds(xs[s], L, "adapted", out=outs[s], workspace=ws),
            "separable_passes": lambda s: dwt.fwd_separable(xs[s], L, out=outs[s], workspace=ws),
            "cdf97_product": lambda s: dwt.fwd_cdf97(xs[s], L, out=outs[s], workspace=ws),
            "cdf97_nonseparable": lambda s: _tiled97(lambda: dwt.fwd_cdf97(xs[s], L, out=outs[s], workspace=ws)),
            "cdf97_separable": lambda s: dwt.fwd_cdf97_separable(xs[s], L, out=outs[s], workspace=ws),
        }
        for name, f in variants.items():
            ms = med(f)
            row[name + "_us"] = round(ms * 1e3, 2)
            row[name + "_Gpx_s"] = round(edge * edge / (ms * 1e-3) / 1e9, 1)
        print(json.dumps(row), flush=True)
        del xs, outs, ws
        torch.cuda.empty_cache()

    edge = 8192
    xs = [synth.image_device(edge, edge, 2 + 100 * s, device=dev) for s in range(2)]
    outs = [torch.empty_like(x) for x in xs]
    ws = torch.empty(dwt.workspace_size(edge, edge, 1), dtype=torch.uint8, device=dev)
    try:
        for seg in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 2048):
            row = {"sweep": "work_item", "edge": edge, "level": 1, "seg_quad_rows": seg}
            for ch in (1, 2, 4):
                dwt.set_tiling(seg, ch)
                ms = med(lambda s: dwt.fwd(xs[s], 1, out=outs[s], workspace=ws))
                row[f"chunk{ch}_us"] = round(ms * 1e3, 2)
            print(json.dumps(row), flush=True)
        dwt.set_tiling(0, 0)
        ms = med(lambda s: dwt.fwd(xs[s], 1, out=outs[s], workspace=ws))
        print(json.dumps({"sweep": "work_item", "edge": edge, "level": 1, "seg_quad_rows": "auto",
                          "auto_us": round(ms * 1e3, 2)}), flush=True)
    finally:
        dwt.set_tiling(0, 0)


if __name__ == "__main__":
    main()
