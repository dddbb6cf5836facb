"""Binocular frame-rate benchmark of the per-frame hot path on one MI355X.

Workload: the synthetic city (1M anchors, 32-dim features, k = 10, octree
LOD 0-10) flown through along a 300-frame rise from 2 m to 300 m, stereo
2048x1080 per eye, IPD 64 mm.  One step = one stereo frame: unified camera,
anchor selection, cache schedule, derivation of the misses, compose,
per-eye projection, binning, sort and blend (inputs resident in HBM).

Prints ONE JSON line (rank 0).  See the design doc for the roofline accounting.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=240)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--form", default="cached-bf16", choices=["plain", "cached", "cached-bf16", "cached-fp8",
                                                               "cached-bf16-learned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-psnr", action="store_true")
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--profile-frames", type=int, default=0, help="only run this many frames (profiling)")
    ap.add_argument("--stats", action="store_true", help="print per-frame counters of every 30th frame to stderr")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus %d is not supported "
                                   "(the path shards by viewer, see DESIGN.md)" % args.gpus}))
        sys.exit(2)
    import torch
    import paper_2502_14938_amd as gs
    import synth

    torch.cuda.set_device(0)
    scene = synth.city_scene()
    traj = synth.city_flythrough(args.frames)
    W, H = synth.CITY_W, synth.CITY_H
    form = args.form
    kw = dict(k=scene.k, max_width=W, max_height=H)
    if form.startswith("cached"):
        kw.update(reuse=True, d_max=10)
    if "bf16" in form:
        kw.update(precision="bf16")
    if "fp8" in form:
        kw.update(precision="fp8")
    r = gs.Renderer(**kw)
    r.load(scene)
    oL = torch.zeros(3, H, W, device="cuda")
    oR = torch.zeros(3, H, W, device="cuda")
    n_frames = len(traj)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        L, R = traj[i % n_frames]
        r.frame(L, R, oL, oR)
    torch.cuda.synchronize()
    r.sync()
    r.reset_cache()
    steps = args.steps if not args.profile_frames else args.profile_frames
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        L, R = traj[i % n_frames]
        ev[i][0].record(stream)
        r.frame(L, R, oL, oR)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r.sync()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    if args.stats:
        r.reset_cache()
        for i in range(n_frames):
            L, R = traj[i]
            r.frame(L, R, oL, oR)
            if i % 30 == 0 or i == n_frames - 1:
                print("frame %d %s" % (i, json.dumps(r.stats())), file=sys.stderr, flush=True)
    total_s = t1 - t0
    fps = steps / total_s
    out = {"metric": "binocular 2K frames/sec and p99 frame latency at PSNR>=40dB vs plain FP32",
           "value": round(fps, 2), "unit": "stereo frames/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": round(1000 * total_s / steps, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if form in ("plain", "cached") else form.split("-")[1],
           "data": "synthetic",
           "config": {"workload": "synthetic city 1M anchors, 300-frame fly-through 2->300 m, stereo 2048x1080",
                      "form": form, "frames": n_frames},
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4), "max": round(float(lat.max()), 4)}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
