"""Throughput of the MI355X volume ray caster on the three-source 256^3 1080p workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: density (lognormal background x cylindrical wake), E and B
(divergence-free sinusoids; chains `length` and `length | mul(2) | pow(0.5)`)
on a 256^3 grid with one guard layer and 256-byte row pitch, trilinear
sampling, step 0.5 voxel, two clipping planes, 8-point transfer functions,
weights in [0.3,1], rendered at 1920x1080 from the 26 neighbour directions of
a cube cell at twice the grid diagonal (fovy 60).  One step = one frame (one
view; steps cycle through the 26 views).  Sources are resident in device
memory before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray samples/sec (Gsamples/s) + frames/s at 1920x1080; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(scene, gpu_counts, row_stride: int, threads: int):
    """The FP64 oracle on every row_stride-th row of the first view, on host threads."""
    import oracle
    rows = np.arange(0, scene.height, row_stride)
    px = np.stack(np.meshgrid(np.arange(scene.width), rows), axis=-1).reshape(-1, 2).astype(np.int32)
    # split the pixel list over threads running the single-threaded oracle
    import threading
    parts = np.array_split(np.arange(px.shape[0]), threads)
    outs = [None] * threads

    def work(k):
        outs[k] = oracle.render_pixels(scene, px[parts[k]])

    t0 = time.perf_counter()
    ts = [threading.Thread(target=work, args=(k,)) for k in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    rec = np.concatenate(outs)
    samples = int(rec["samples"].sum())
    g = gpu_counts[px[:, 1], px[:, 0]].astype(np.int64)
    agree = float(np.mean(g == rec["samples"]))
    return dict(value=samples / dt / 1e9, unit="Gsamples/s", cores=threads, kind="oracle",
                sample=f"every {row_stride}th row of view 0 ({px.shape[0]} pixels, {samples} samples, "
                       f"{dt:.1f} s wall on {threads} threads); per-pixel sample counts equal to the GPU's "
                       f"on {agree * 100:.2f}% of them")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=104)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--views", type=int, default=26)
    ap.add_argument("--cpu-row-stride", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the ray caster has no multi-GPU path "
              f"in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, Context, device
    from scenes import configs

    torch.cuda.set_device(0)
    log(f"bench: generating pic3 {args.n}^3 {args.dtype} {args.width}x{args.height}")
    sc = configs.pic3(n=args.n, width=args.width, height=args.height, dtype=args.dtype)
    stream = torch.cuda.current_stream()
    ctx = Context(device=0, stream=stream)
    vol = device.upload_volume(ctx, sc, 0)
    img = device.new_image(sc)
    cnt = device.new_counts(sc)
    views = configs.views26()[: args.views]
    scenes_v = [sc.with_(camera=configs.orbit_camera(sc.dims, v)) for v in views]
    jobs = [device.render_job(s, 0, img) for s in scenes_v]
    log("bench: counting samples per view (untimed)")
    samples = []
    hit = []
    for s in scenes_v:
        ctx.render([device.render_job(s, 0, img, cnt)])
        c = cnt.to(torch.int64)
        samples.append(int(c.sum().item()))
        hit.append(float((c > 0).float().mean().item()))
    counts_view0 = None
    ctx.render([device.render_job(scenes_v[0], 0, img, cnt)])
    counts_view0 = cnt.cpu().numpy()
    log(f"bench: samples/frame mean {np.mean(samples):.4g} (min {min(samples)}, max {max(samples)}); "
        f"hit fraction {np.mean(hit):.3f}")

    for k in range(args.warmup):
        ctx.render([jobs[k % len(jobs)]], ASYNC)
    torch.cuda.synchronize()
    ctx.timing()    # discard warm-up timings

    # timed region: K frames cycling through the views
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        ctx.render([jobs[k % len(jobs)]], ASYNC | TIMING)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    kernel_ms, n_kernels = ctx.timing()
    frame_ms = np.array([a.elapsed_time(b) for a, b in ev])
    total_samples = sum(samples[k % len(jobs)] for k in range(args.steps))
    gsps = total_samples / elapsed / 1e9
    per_view = np.zeros(len(views))
    for k in range(args.steps):
        per_view[k % len(jobs)] += frame_ms[k]
    reps = np.bincount(np.arange(args.steps) % len(jobs), minlength=len(jobs))
    per_view = per_view / np.maximum(reps, 1)
    log(f"bench: {args.steps} frames in {elapsed * 1e3:.1f} ms -> {gsps:.2f} Gsamples/s; kernel avg "
        f"{kernel_ms / max(n_kernels, 1):.3f} ms")

    # roofline of the ray-casting kernel: every source byte once plus the image, per launch
    field_bytes = sum(s.field_bytes() for s in sc.sources)
    image_bytes = sc.width * sc.height * 16
    algo_bytes = field_bytes + image_bytes
    kavg_s = kernel_ms / max(n_kernels, 1) / 1e3
    achieved = algo_bytes / kavg_s / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    kernel="raycast_kernel", kernel_avg_ms=round(kavg_s * 1e3, 4),
                    algorithmic_bytes_per_launch=algo_bytes)

    out = dict(metric=METRIC, value=round(gsps, 3), unit="Gsamples/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(elapsed * 1e3 / args.steps, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype=args.dtype, data="synthetic",
               config=dict(workload=f"pic3: density+E+B {args.n}^3, 1 guard layer, trilinear, step 0.5, "
                                    f"2 clip planes, {args.width}x{args.height}, {len(views)} views",
                           grid=args.n, width=args.width, height=args.height, sources=3,
                           storage=args.dtype, views=len(views)),
               fps=round(args.steps / elapsed, 2),
               latency_ms=dict(p50=round(float(np.percentile(frame_ms, 50)), 4),
                               p99=round(float(np.percentile(frame_ms, 99)), 4)),
               views_ms=dict(avg=round(float(per_view.mean()), 4), min=round(float(per_view.min()), 4),
                             max=round(float(per_view.max()), 4)),
               samples_per_frame=int(np.mean(samples)),
               roofline=roofline)
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        log(f"bench: CPU oracle baseline on {threads} threads")
        out["cpu_baseline"] = cpu_baseline(scenes_v[0], counts_view0, args.cpu_row_stride, threads)
    del vol
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
