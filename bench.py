"""Throughput of the MI355X volume ray caster on the three-source 256^3 1080p workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload: density (lognormal background x cylindrical wake), E and
B (divergence-free sinusoids; chains `length` and `length | mul(2) | pow(0.5)`)
on a 256^3 grid with one guard layer and 256-byte row pitch, trilinear
sampling, step 0.5 voxel, two clipping planes, 8-point transfer functions,
weights in [0.3,1], rendered at 1920x1080 from the 26 neighbour directions of
a cube cell at twice the grid diagonal (fovy 60).  One step = one frame (one
view; steps cycle through the 26 views).  Sources are resident in device
memory before timing starts; `value` counts the scan points composited
(counted once per view by the kernel's counting variant, untimed).

Also reported (not the headline): the same scene with FP16 and BF16 storage
and in iso-surface mode, the RGBA8 frame encode, a field simulation on
128^3 rendered in situ every step and every 10th step, the 64-sub-volume
batch in one persistent hipGraph launch, and a short run of the
continuous-batching server on a resident 512x512x256 volume.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray samples/sec (Gsamples/s) + frames/s at 1920x1080; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (it counts packed FP32, two FMAs per lane and cycle)
FP32_VALU_PEAK_TFLOPS = 157.3
# the same chip without packed FP32 (which this build does not use): 256 CUs x 4 SIMDs
# x 16 lanes x 2 FLOP per FMA x 2.4 GHz
FP32_VALU_NONPACKED_TFLOPS = 78.6
# per scan point, 3 sources, trilinear: position 11, cell weights 6, per source
# 7 lerps (21) + classification (12) + weighted mix (8), front-to-back composite
# and termination test 10
FLOPS_PER_SAMPLE = 150
TUNED = os.path.join(ROOT, "paper_1611_09048_amd", "tuned_gfx950.json")
# candidates the bench tunes over when its cache has no entry
QUICK = dict(lanes=(4, 8, 16, 32), wave_ws=(2, 4, 8, 16), waves_xs=(1, 2, 4), unrolls=(1,), min_waves=(0, 4))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "pic3_256_1080p_frame_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1611_09048_amd", "csrc", "raycast.hip")
VIEW_SAMPLES = os.path.join(ROOT, "tests", "golden", "pic3_256_1080p_view_samples.json")


def measured_counters(shape):
    """Fields of the committed counter summary of the headline frame (HBM bytes
    per frame and per kernel, L2 hit rates), or None when the kernel source or
    the launch's tile shape `shape` differ from the ones the counters were
    taken with."""
    import hashlib
    try:
        text = open(COUNTERS).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith(("#", "|", " ", "-")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel source sha256") != src or fields.get("tile shape") != ",".join(map(str, shape)):
        return None
    return fields


def measured_traffic(shape):
    """HBM bytes (fetched + written, calibrated) per headline frame from the counters, or None."""
    f = measured_counters(shape)
    if f is None or "traffic_bytes_per_frame" not in f:
        return None
    return int(f["traffic_bytes_per_frame"])


def measured_l2_hit_rate(shape):
    """L2 hit rate per kernel of the headline frame from the counters, or None."""
    f = measured_counters(shape)
    if f is None:
        return None
    out = {k[len("l2_hit_rate "):]: float(v) for k, v in f.items() if k.startswith("l2_hit_rate ")}
    return out or None


def oracle_view_samples(n, width, height, dtype):
    """The oracle's exact scan-point counts of the 26 views (a committed file that a
    script calling only the oracle wrote), for the FP32 headline size; else None."""
    if (n, width, height, dtype) != (256, 1920, 1080, "f32"):
        return None
    try:
        with open(VIEW_SAMPLES) as f:
            return json.load(f)
    except OSError:
        return None


def host_cpu():
    """(model name, cores this process may run on)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(scene, gpu_img, gpu_counts, threads: int, row_stride_all: int = 4, row_stride_one: int = 16,
                 storage_images=None):
    """The FP64 oracle timed on host cores: one thread on every row_stride_one-th row of
    view 0, then `threads` threads on every row_stride_all-th row.  Each run's pixels are
    also compared with the GPU frame (RGBA within 2e-3 plus the oracle's allowance, and
    the sample counts); storage_images ({storage: GPU frame of view 0 rendered from the
    fields stored that way}) get their per-channel max and RMS error against the same
    oracle pixels of the FP32 fields."""
    import oracle
    records = {}

    def run(stride, n_threads):
        rows = np.arange(0, scene.height, stride)
        px = np.stack(np.meshgrid(np.arange(scene.width), rows), axis=-1).reshape(-1, 2).astype(np.int32)
        parts = np.array_split(np.arange(px.shape[0]), n_threads)
        outs = [None] * n_threads

        def work(k):
            outs[k] = oracle.render_pixels(scene, px[parts[k]])

        t0 = time.perf_counter()
        ts = [threading.Thread(target=work, args=(k,)) for k in range(n_threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        dt = time.perf_counter() - t0
        rec = np.concatenate(outs)
        records[stride] = (px, rec)
        g = gpu_img[px[:, 1], px[:, 0]].astype(np.float64)
        diff = np.abs(g - rec["rgba"])
        within = diff <= 2e-3 + rec["allowance"][:, None]
        counts_equal = gpu_counts[px[:, 1], px[:, 0]].astype(np.int64) == rec["samples"]
        samples = int(rec["samples"].sum())
        return dict(msamples_per_s=round(samples / dt / 1e6, 4), seconds=round(dt, 2), pixels=int(px.shape[0]),
                    samples=samples, threads=n_threads, rows=f"every {stride}th row",
                    max_abs_diff_rgba=float(diff.max()), pixels_within_bound=float(np.mean(within.all(axis=1))),
                    counts_equal=float(np.mean(counts_equal)),
                    flagged_pixels=int((rec["flags"] > 0).sum()))

    model, visible = host_cpu()
    one = run(row_stride_one, 1)
    log(f"bench: oracle on 1 thread {one}")
    allc = run(row_stride_all, threads)
    log(f"bench: oracle on {threads} threads {allc}")
    px, rec = records[row_stride_all]
    errors = {}
    for name, img in (storage_images or {}).items():
        d = img[px[:, 1], px[:, 0]].astype(np.float64) - rec["rgba"]
        errors[name] = dict(max=[float(v) for v in np.abs(d).max(axis=0)],
                            rms=[float(v) for v in np.sqrt((d * d).mean(axis=0))])
    return dict(value=round(allc["msamples_per_s"] / 1e3, 6), unit="Gsamples/s", cores=threads, kind="oracle",
                storage_error_vs_oracle_of_fp32_fields=errors or None,
                sample=(f"view 0 of the headline frame: {allc['rows']} ({allc['pixels']} pixels, "
                        f"{allc['samples']} samples, {allc['seconds']} s on {threads} threads); single thread on "
                        f"{one['rows']} ({one['samples']} samples, {one['seconds']} s)"),
                cpu_model=model, host_cores_visible=visible, single_thread_msamples_per_s=one["msamples_per_s"],
                all_cores_msamples_per_s=allc["msamples_per_s"],
                parity_vs_gpu=dict(max_abs_diff_rgba=max(one["max_abs_diff_rgba"], allc["max_abs_diff_rgba"]),
                                   pixels_within_bound=min(one["pixels_within_bound"], allc["pixels_within_bound"]),
                                   counts_equal=min(one["counts_equal"], allc["counts_equal"]),
                                   pixels=allc["pixels"], flagged_pixels=allc["flagged_pixels"]))


FORCED_SHAPE = None


def apply_tuning(ctx, key_sig, classes, time_jobs, retune=False):
    """Set the tile shape of `classes` from the cache, tuning (one shape for all) when missing."""
    from paper_1611_09048_amd import autotune
    if FORCED_SHAPE is not None:
        for c in classes:
            ctx.set_tile_shape(c, *FORCED_SHAPE)
        return FORCED_SHAPE
    cache = autotune.load_cache(TUNED)
    key = autotune.cache_key("gfx950", "+".join(map(str, classes)), key_sig)
    if key in cache and not retune:
        best = tuple(cache[key])
    else:
        times = {}
        for cand in autotune.candidates(**QUICK):
            for c in classes:
                ctx.set_tile_shape(c, *cand)
            times[cand] = time_jobs()
        best = autotune.pick(times)
        log(f"bench: tuned {key}: {best} {times[best]:.4f} ms (of {len(times)} candidates)")
        cache[key] = list(best)
        try:
            autotune.save_cache(TUNED, cache)
        except OSError:
            pass
    for c in classes:
        ctx.set_tile_shape(c, *best)
    return best


def frames(ctx, sc, steps, warmup, view_reps=0, log_prefix=""):
    """Time `steps` frames cycling through the 26 views back to back (throughput), the
    same frames each between two events (latency), then (view_reps > 0) each view
    view_reps times in a pass of its own; returns a dict of results.  The context
    enqueues on torch's current stream, so the events recorded there around each
    render bracket all of its device work (derive, set-up and ray-casting passes)."""
    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, device
    from scenes import configs
    stream = torch.cuda.current_stream()
    vol = device.upload_volume(ctx, sc, 0)
    img = device.new_image(sc)
    cnt = device.new_counts(sc)
    views = configs.views26()
    scenes_v = [sc.with_(camera=configs.orbit_camera(sc.dims, v)) for v in views]
    jobs = [device.render_job(s, 0, img) for s in scenes_v]

    def time_jobs():
        ctx.render([jobs[0]])
        ctx.timing()
        for j in (jobs[0], jobs[8], jobs[13], jobs[20]):
            ctx.render([j], TIMING)
        ms, n = ctx.timing()
        return ms / n

    from paper_1611_09048_amd import autotune
    sig = f"pic3:{sc.sources[0].dtype}"
    shape = apply_tuning(ctx, sig, [autotune.size_class(sc.width, sc.height)], time_jobs)
    samples, hit = [], []
    for s in scenes_v:
        ctx.render([device.render_job(s, 0, img, cnt)])
        c = cnt.to(torch.int64)
        samples.append(int(c.sum().item()))
        hit.append(float((c > 0).float().mean().item()))
    ctx.render([device.render_job(scenes_v[0], 0, img, cnt)])
    counts_view0 = cnt.cpu().numpy()
    image_view0 = img.cpu().numpy()
    # what clipping and early termination remove (view 0, untimed)
    ctx.render([device.render_job(scenes_v[0], 0, img, cnt, ert_threshold=2.0)])
    no_ert = int(cnt.to(torch.int64).sum().item())
    ctx.render([device.render_job(scenes_v[0].with_(clip=[]), 0, img, cnt, ert_threshold=2.0)])
    no_clip_no_ert = int(cnt.to(torch.int64).sum().item())
    ctx.render([device.render_job(scenes_v[0], 0, img, cnt)])
    removed = dict(samples_view0=int(counts_view0.sum()), without_termination=no_ert,
                   without_clip_or_termination=no_clip_no_ert,
                   clipped_fraction=round(1.0 - no_ert / max(no_clip_no_ert, 1), 4),
                   terminated_fraction=round(1.0 - int(counts_view0.sum()) / max(no_ert, 1), 4))
    # the numerator: the oracle's exact counts where they are on file, else the GPU's
    ref = oracle_view_samples(sc.dims[0], sc.width, sc.height, sc.sources[0].dtype) if sc.dims[0] == sc.dims[1] == \
        sc.dims[2] else None
    gpu_samples = list(samples)
    counted_by = "gpu counting variant"
    if ref is not None and len(ref["samples"]) == len(views):
        samples = [int(v) for v in ref["samples"]]
        counted_by = "oracle"
    log(f"bench:{log_prefix} samples/frame mean {np.mean(samples):.4g} (min {min(samples)}, max {max(samples)}, "
        f"counted by the {counted_by}); hit fraction {np.mean(hit):.3f}; tile shape {shape}")
    for k in range(warmup):
        ctx.render([jobs[k % len(jobs)]], ASYNC)
    torch.cuda.synchronize()
    ctx.timing()
    # throughput: the frames back to back, bracketed by device synchronizations and
    # two events on the render stream, with no marker between frames (an event
    # marker between two launches costs device time of its own, ~9 us per frame
    # with two); the events' span over the K frames is the mean device time of a
    # frame in the timed region
    span = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    span[0].record(stream)
    for k in range(steps):
        ctx.render([jobs[k % len(jobs)]], ASYNC)
    span[1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    frame_avg_ms = span[0].elapsed_time(span[1]) / steps
    # latency: the same frames again, each between two events on the render stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record(stream)
        ctx.render([jobs[k % len(jobs)]], ASYNC)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    frame_ms = np.array([a.elapsed_time(b) for a, b in ev])
    # the ray-casting kernel alone, bracketed by the library's events (which add a
    # marker between the passes, so not inside the timed frames): one pass over the views
    ctx.timing()
    for j in jobs:
        ctx.render([j], ASYNC | TIMING)
    torch.cuda.synchronize()
    kernel_ms, n_kernels = ctx.timing()
    total = sum(samples[k % len(jobs)] for k in range(steps))
    out = dict(gsps=total / elapsed / 1e9, elapsed=elapsed, kernel_ms=kernel_ms / max(n_kernels, 1),
               frame_ms=frame_ms, frame_avg_ms=frame_avg_ms, samples=samples, gpu_samples=gpu_samples, counted_by=counted_by, shape=shape,
               counts_view0=counts_view0, image_view0=image_view0, scene_v0=scenes_v[0],
               field_bytes=sum(s.field_bytes() for s in sc.sources), removed=removed,
               image_bytes=sc.width * sc.height * 16, oracle_ref=ref)
    log(f"bench:{log_prefix} {steps} frames in {elapsed * 1e3:.1f} ms -> {out['gsps']:.2f} Gsamples/s; "
        f"frame p50 {np.median(frame_ms):.4f} ms (device, events); ray-casting kernel avg {out['kernel_ms']:.4f} ms")
    if view_reps > 0:
        # each view on its own: one untimed frame, then view_reps timed ones, back to back
        vev = []
        for v in range(len(views)):
            ctx.render([jobs[v]], ASYNC)
            for _ in range(view_reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ctx.render([jobs[v]], ASYNC)
                b.record(stream)
                vev.append((v, a, b))
        torch.cuda.synchronize()
        per = [[] for _ in views]
        for v, a, b in vev:
            per[v].append(a.elapsed_time(b))
        med = np.array([float(np.median(p)) for p in per])
        gs = np.array(samples, dtype=np.float64) / (med / 1e3) / 1e9
        out["views"] = dict(reps=view_reps, frame_ms=dict(avg=round(float(med.mean()), 4), min=round(float(med.min()), 4),
                                                          max=round(float(med.max()), 4)),
                            gsamples_per_s=dict(avg=round(float(gs.mean()), 3), min=round(float(gs.min()), 3),
                                                max=round(float(gs.max()), 3)),
                            slowest_over_fastest=round(float(med.max() / med.min()), 3),
                            per_view_ms=[round(float(m), 4) for m in med],
                            samples_per_view=[int(x) for x in samples])
        log(f"bench:{log_prefix} views {out['views']['frame_ms']} ms, {out['views']['gsamples_per_s']} Gsamples/s")
    del vol
    return out


def bricks8(ctx, sc, reps: int = 5):
    """One GPU's share of the sort-last design: the 256^3 volume as 8 bricks of 128^3 (one per
    rank), each rendered on its own at 1080p on the global step grid, then the 8-layer
    over-composite. Reports the mean brick render (ray-casting kernel) and the composite time."""
    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, device
    from scenes import make_source
    half = sc.dims[0] // 2
    vols, layers, depths, jobs = [], [], [], []
    for k, (x, y, z) in enumerate([(x, y, z) for x in (0, half) for y in (0, half) for z in (0, half)]):
        srcs = []
        for s in sc.sources:
            v = s.values[z:z + half + 2, y:y + half + 2, x:x + half + 2]    # global index i -> array i + 1
            srcs.append(make_source(s.name, v.astype(np.float32) if s.dtype == "f32" else v, dtype=s.dtype,
                                    guard=1, chain=s.chain, weight=s.weight, tf=s.tf))
        bs = sc.with_(dims=(half, half, half), sources=srcs)
        vols.append(device.upload_volume(ctx, bs, 240 + k))
        img = device.new_image(sc)
        dep = torch.empty((sc.height, sc.width), device="cuda")
        layers.append(img)
        depths.append(dep)
        jobs.append(device.render_job(sc, 240 + k, img, brick_origin=(x, y, z), global_dims=sc.dims,
                                      out_depth=dep.data_ptr(), ert_threshold=2.0))
    out = device.new_image(sc)
    for j in jobs:
        ctx.render([j])
    torch.cuda.synchronize()
    ctx.timing()
    for _ in range(reps):
        for j in jobs:
            ctx.render([j], ASYNC | TIMING)
    torch.cuda.synchronize()
    ms, n = ctx.timing()
    lp, dp = [l.data_ptr() for l in layers], [d.data_ptr() for d in depths]
    ctx.composite(lp, dp, sc.width, sc.height, out.data_ptr())
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    a.record(stream)
    for _ in range(reps):
        ctx.composite(lp, dp, sc.width, sc.height, out.data_ptr(), 1)
    b.record(stream)
    torch.cuda.synchronize()
    res = dict(bricks=8, brick_dims=[half] * 3, brick_raycast_kernel_ms=round(ms / max(n, 1), 4),
               composite_ms=round(a.elapsed_time(b) / reps, 4))
    log(f"bench: bricks8 {res}")
    del vols
    return res


def served_readback(ctx, reps: int = 10, n: int = 512, depth: int = 256):
    """A served 1920x1080 request on the frozen resident volume, from submission to the image in
    host memory: as RGBA32F (33 MB over PCIe), as RGBA8 (8 MB) and as JPEG (quality 90)."""
    import torch
    from paper_1611_09048_amd import device
    from scenes import configs
    dims = (n, n, depth)
    sc = configs.pic3(dims=dims, width=1920, height=1080)
    vol = device.upload_volume(ctx, sc, 201)
    ctx.freeze_volume(201)
    job = device.render_job(sc, 201, device.new_image(sc))
    f32 = np.empty((sc.height, sc.width, 4), np.float32)
    u8 = np.empty((sc.height, sc.width, 4), np.uint8)
    reads = {"rgba32f": lambda t: ctx.read_image(t, f32),
             "rgba8": lambda t: ctx.read_image_rgba8(t, u8, (1.0, 1.0, 1.0)),
             "jpeg": lambda t: ctx.read_image_jpeg(t, sc.width, sc.height, 90, (1.0, 1.0, 1.0))}
    res = {}
    for name, read in reads.items():
        for k in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = ctx.submit(job)
            out = read(t)
            dt = time.perf_counter() - t0
            ctx.release(t)
            if k == 0:
                continue                     # first call: buffers and graphs are set up
            res.setdefault(name, []).append(dt * 1e3)
        res[name] = round(float(np.median(res[name])), 3)
    res["jpeg_bytes"] = len(out)
    log(f"bench: served readback (ms, submit to host image) {res}")
    del vol
    return res


def batch64(ctx, steps):
    """The 64-sub-volume workload as one batched launch (hipGraph replay)."""
    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, autotune, device
    from scenes import configs
    scs = configs.batch64()
    vols = [device.upload_volume(ctx, sc, vid) for vid, sc in enumerate(scs)]
    imgs = [device.new_image(sc) for sc in scs]
    cnts = [device.new_counts(sc) for sc in scs]
    jobs = [device.render_job(sc, vid, imgs[vid]) for vid, sc in enumerate(scs)]
    classes = sorted({autotune.size_class(sc.width, sc.height) for sc in scs})

    def time_jobs():
        ctx.render(jobs)
        ctx.timing()
        for _ in range(2):
            ctx.render(jobs, TIMING)
        ms, n = ctx.timing()
        return ms / n

    shape = apply_tuning(ctx, "batch64:f32x1", classes, time_jobs)
    # one launch shares the kernel variant; each size class then takes its own tile shape
    cache = autotune.load_cache(TUNED)
    n_before = len(cache)
    per_class = autotune.refine_per_class(ctx, classes, shape, time_jobs, cache=cache, sig="batch64:f32x1:class",
                                          log=log)
    if len(cache) != n_before:
        try:
            autotune.save_cache(TUNED, cache)
        except OSError:
            pass
    ctx.render([device.render_job(sc, vid, imgs[vid], cnts[vid]) for vid, sc in enumerate(scs)])
    samples = int(sum(int(c.to(torch.int64).sum().item()) for c in cnts))
    ctx.render(jobs, ASYNC)
    torch.cuda.synchronize()
    ctx.timing()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.render(jobs, ASYNC | TIMING)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = ctx.timing()
    res = dict(jobs=len(scs), samples_per_batch=samples, launch_ms=round(el * 1e3 / steps, 4),
               graph_ms=round(ms / max(n, 1), 4), gsamples_per_s=round(samples * steps / el / 1e9, 3),
               jobs_per_s=round(len(scs) * steps / el, 1), tile_shape=list(shape),
               tile_shape_per_class={str(c): list(v) for c, v in per_class.items()},
               rays=int(sum(sc.width * sc.height for sc in scs)))
    log(f"bench: batch64 {res}")
    del vols
    return res


def serving(ctx, duration: float, rate: float, n: int = 512, depth: int = 256, freeze: bool = True):
    """Continuous-batching server on a resident n x n x depth three-source volume (frozen: its
    chains evaluated once per voxel when it is loaded, as a server of a fixed data set would)."""
    from paper_1611_09048_amd import device, serve
    from scenes import configs
    dims = (n, n, depth)
    vol_scene = configs.pic3(dims=dims, width=16, height=16)
    vol = device.upload_volume(ctx, vol_scene, 200)
    if freeze:
        ctx.freeze_volume(200)
    ex = serve.DeviceExecutor(ctx, vol, dims)
    srv = serve.Server(ex, time.perf_counter, max_batch=16, max_batches_in_flight=3)
    reqs = configs.serving_requests(11, dims, n_clients=4, rate_per_client=rate / 4, duration=duration,
                                    base_tfs=[s.tf for s in vol_scene.sources])
    dur = serve.run(srv, reqs, time.perf_counter, make_job=serve.job_from_request)
    out = srv.summary(dur)
    out.update(volume=list(dims), offered_rate=rate, requests=len(reqs), frozen=freeze)
    log(f"bench: serving {out}")
    del vol
    def rnd(v):
        if isinstance(v, float):
            return round(v, 4)
        if isinstance(v, dict):
            return {k: rnd(x) for k, x in v.items()}
        return v
    return {k: rnd(v) for k, v in out.items()}


def iso_frames(ctx, n: int, width: int, height: int, steps: int = 26):
    """The headline scene in iso-surface mode: density surface at 1.0, |E| surface at 0.2."""
    import dataclasses
    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, device
    from scenes import configs
    sc = configs.pic3(n=n, width=width, height=height)
    sc = sc.with_(mode="iso", sources=[dataclasses.replace(s, iso=v) for s, v in
                                       zip(sc.sources, (1.0, 0.2, float("nan")))])
    vol = device.upload_volume(ctx, sc, 220)
    img, cnt = device.new_image(sc), device.new_counts(sc)
    views = [sc.with_(camera=configs.orbit_camera(sc.dims, v)) for v in configs.views26()]
    samples, surf = [], []
    for v in views:
        ctx.render([device.render_job(v, 220, img, cnt)])
        samples.append(int(cnt.to(torch.int64).sum().item()))
        surf.append(float((img[..., 3] == 1.0).float().mean().item()))
    jobs = [device.render_job(v, 220, img) for v in views]
    ctx.render(jobs[:1])
    torch.cuda.synchronize()
    ctx.timing()
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.render([jobs[k % 26]], ASYNC | TIMING)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, nk = ctx.timing()
    total = sum(samples[k % 26] for k in range(steps))
    res = dict(gsamples_per_s=round(total / el / 1e9, 3), fps=round(steps / el, 2),
               kernel_ms=round(ms / max(nk, 1), 4), samples_per_frame=int(np.mean(samples)),
               surface_pixel_fraction=round(float(np.mean(surf)), 4))
    log(f"bench: iso {res}")
    del vol
    return res


def encode(ctx, width: int, height: int, reps: int = 50):
    """RGBA32F -> RGBA8 frame encode over a background; bytes = 16 read + 4 written per pixel."""
    import torch
    img = torch.rand((height, width, 4), device="cuda")
    out = torch.empty((height, width, 4), dtype=torch.uint8, device="cuda")
    ctx.encode_rgba8(img.data_ptr(), width, height, out.data_ptr(), (1.0, 1.0, 1.0))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    a.record(stream)
    for _ in range(reps):
        ctx.encode_rgba8(img.data_ptr(), width, height, out.data_ptr(), (1.0, 1.0, 1.0), 1)
    b.record(stream)
    torch.cuda.synchronize()
    us = a.elapsed_time(b) * 1e3 / reps
    res = dict(us_per_frame=round(us, 2), gb_per_s=round(width * height * 20 / (us * 1e-6) / 1e9, 1))
    log(f"bench: encode {res}")
    return res


def jpeg_frames(ctx, sc, reps: int = 20, quality: int = 90):
    """JPEG compression of a rendered frame (over white, quality 90) and of a noise frame, wall clock per call."""
    import torch
    from paper_1611_09048_amd import device
    vol = device.upload_volume(ctx, sc, 9)
    img = device.new_image(sc)
    ctx.render([device.render_job(sc, 9, img)])
    w, h = sc.width, sc.height
    rgba8 = torch.empty((h, w, 4), dtype=torch.uint8, device="cuda")
    ctx.encode_rgba8(img.data_ptr(), w, h, rgba8.data_ptr(), (1.0, 1.0, 1.0))
    noise = torch.randint(0, 256, (h, w, 4), dtype=torch.uint8, device="cuda")
    res = dict(quality=quality)
    for name, t in (("frame", rgba8), ("noise", noise)):
        b = ctx.encode_jpeg(t.data_ptr(), w, h, quality)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.encode_jpeg(t.data_ptr(), w, h, quality)
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[name] = dict(ms_per_frame=round(ms, 3), bytes=len(b), bits_per_pixel=round(8 * len(b) / (w * h), 3),
                         mpixel_per_s=round(w * h / (ms * 1e3), 1))
    log(f"bench: jpeg {res}")
    del vol
    return res


def insitu_run(ctx, n: int, width: int, height: int, steps: int = 40):
    """A field simulation on the same stream, rendered every n-th step (zero-copy sources)."""
    import torch
    from paper_1611_09048_amd import binding, insitu
    from scenes import configs
    sim = insitu.FieldSimulation(n=n, seed=7)
    r = insitu.InSituRenderer(ctx, sim, volume_id=230)
    img = torch.empty((height, width, 4), device="cuda")
    views = configs.views26()
    dims = (n, n, n)

    def make_desc(frame):
        cam = configs.orbit_camera(dims, views[frame % 26])
        return binding.render_desc(volume_id=230, width=width, height=height, eye=cam.eye, center=cam.center,
                                   up=cam.up, fovy_deg=cam.fovy_deg, step=0.5, interpolation=binding.TRILINEAR,
                                   out_rgba=img.data_ptr())

    r.render(make_desc(0))
    alone = r.run(steps, 0, make_desc)
    res = dict(grid=n, width=width, height=height, steps=steps, sim_ms_per_step=round(alone.total_s * 1e3 / steps, 3))
    for every in (1, 10):
        st = r.run(steps, every, make_desc)
        res[f"every_{every}"] = dict(frames=st.frames, ms_per_step=round(st.total_s * 1e3 / steps, 3),
                                     render_ms_per_frame=round(st.render_s * 1e3 / max(st.frames, 1), 3),
                                     render_share=round(st.overhead, 4))
    log(f"bench: in situ {res}")
    return res


def copy_probe(ctx_unused, mib: int = 512, reps: int = 3):
    """A plain device copy of known size, for normalizing rocprof byte counters."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    return dict(bytes_read=x.numel() * 4, bytes_written=y.numel() * 4, kernels=reps)


def check_frame_timing(frame_ms, kernel_ms):
    """Frame events must bracket the ray-casting kernel they contain: a frame shorter
    than its kernel means the events were recorded on another stream."""
    if float(np.min(frame_ms)) < kernel_ms * 0.98:
        raise RuntimeError(f"frame events ({float(np.min(frame_ms)):.4f} ms) shorter than the ray-casting kernel "
                           f"({kernel_ms:.4f} ms): they do not bracket the render")


def rooflines(frame_ms, kernel_ms, algo_bytes, samples_per_frame, shape=(), frame_time=None):
    """(HBM roofline of the whole frame, ALU roofline of the ray-casting kernel).

    HBM: every stored source byte and the image once (the frame's algorithmic
    bytes) over the mean device time of a frame (the mean of frame_ms), against
    8 TB/s.  ALU: the method's FLOPs per scan point over the kernel's mean
    duration, against the published FP32 vector peak (and the non-packed peak
    this build runs at)."""
    frame_ms = np.asarray(frame_ms, dtype=np.float64)
    check_frame_timing(frame_ms, kernel_ms)
    mean_ms = float(frame_ms.mean())
    gbs = algo_bytes / (mean_ms / 1e3) / 1e9
    if gbs > HBM_PEAK_GBS:
        raise RuntimeError(f"{gbs:.0f} GB/s of algorithmic bytes is above the HBM peak: the frame time is wrong")
    hbm = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
               traffic=measured_traffic(shape), l2_hit_rate=measured_l2_hit_rate(shape),
               scope="one frame: derive_kernel, prepass_kernel and raycast_kernel, one stream",
               algorithmic_bytes_per_frame=int(algo_bytes), frame_ms_mean=round(mean_ms, 4))
    if frame_time:
        hbm["frame_time"] = frame_time
    flops = FLOPS_PER_SAMPLE * samples_per_frame
    tf = flops / (kernel_ms / 1e3) / 1e12
    alu = dict(bound="alu", kernel="raycast_kernel", achieved=round(tf, 2), peak=FP32_VALU_PEAK_TFLOPS,
               unit="TFLOP/s", frac=round(tf / FP32_VALU_PEAK_TFLOPS, 4), peak_nonpacked=FP32_VALU_NONPACKED_TFLOPS,
               frac_nonpacked=round(tf / FP32_VALU_NONPACKED_TFLOPS, 4), kernel_avg_ms=round(kernel_ms, 4),
               flops_per_sample=FLOPS_PER_SAMPLE, algorithmic_flops_per_launch=int(flops))
    return hbm, alu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=104)
    ap.add_argument("--warmup", type=int, default=52)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--cpu-row-stride", type=int, default=4)
    ap.add_argument("--view-reps", type=int, default=5, help="timed frames per view in the 26-view pass (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--jpeg-only", action="store_true",
                    help="only compress the view-0 frame and a noise frame to JPEG (for profiling); prints that result")
    ap.add_argument("--batch64-only", action="store_true",
                    help="only the batch of 64 sub-volumes, --steps batches (for profiling); prints that result")
    ap.add_argument("--shape", default="", help="wave_w,waves_x,unroll,lanes,min_waves instead of the tuned shape")
    args = ap.parse_args()
    if args.shape:
        global FORCED_SHAPE
        FORCED_SHAPE = tuple(int(v) for v in args.shape.split(","))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): every job of this ray caster is "
              f"rendered by one GPU; the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_09048_amd import Context
    from scenes import configs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = Context(device=0, stream=stream, mem_budget=4 << 30)
    if args.copy_probe:
        log("bench: copy probe", copy_probe(ctx))
    if args.batch64_only:
        print(json.dumps(dict(batch64=batch64(ctx, args.steps))), flush=True)
        ctx.close()
        return
    log(f"bench: generating pic3 {args.n}^3 {args.dtype} {args.width}x{args.height}")
    sc = configs.pic3(n=args.n, width=args.width, height=args.height, dtype=args.dtype)
    if args.jpeg_only:
        print(json.dumps(dict(jpeg=jpeg_frames(ctx, sc, reps=args.steps))), flush=True)
        ctx.close()
        return
    fr = frames(ctx, sc, args.steps, args.warmup, view_reps=args.view_reps)
    roofline, roofline_alu = rooflines([fr["frame_avg_ms"]], fr["kernel_ms"], fr["field_bytes"] + fr["image_bytes"],
                                       float(np.mean(fr["samples"])), fr["shape"],
                                       frame_time="events on the render stream around the K timed frames, span / K")
    out = dict(metric=METRIC, value=round(fr["gsps"], 3), unit="Gsamples/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(fr["elapsed"] * 1e3 / args.steps, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype=args.dtype, data="synthetic",
               config=dict(workload=f"pic3: density+E+B {args.n}^3, 1 guard layer, trilinear, step 0.5, "
                                    f"2 clip planes, {args.width}x{args.height}, 26 views",
                           grid=args.n, width=args.width, height=args.height, sources=3, storage=args.dtype,
                           views=26, tile_shape=list(fr["shape"])),
               fps=round(args.steps / fr["elapsed"], 2),
               latency_ms=dict(p50=round(float(np.percentile(fr["frame_ms"], 50)), 4),
                               p99=round(float(np.percentile(fr["frame_ms"], 99)), 4),
                               what="device time of one frame (derive, set-up and ray casting) from events on "
                                    "the render stream, in a pass of its own after the timed one"),
               samples_per_frame=int(np.mean(fr["samples"])), samples_counted_by=fr["counted_by"],
               sample_reduction_view0=fr["removed"], roofline=roofline, roofline_raycast_alu=roofline_alu)
    if "views" in fr:
        out["views"] = fr["views"]
    if fr["oracle_ref"] is not None:
        g, o = np.array(fr["gpu_samples"]), np.array(fr["samples"])
        out["samples_gpu_vs_oracle"] = dict(max_rel_diff=float(np.max(np.abs(g - o) / o)),
                                            max_abs_diff=int(np.max(np.abs(g - o))),
                                            oracle_count_slack_max=int(max(fr["oracle_ref"]["count_slack"])))
    storage_images = {args.dtype: fr["image_view0"]}
    if not args.no_extras:
        extras = {}
        for dt in ("f16", "bf16"):
            if dt == args.dtype:
                continue
            s2 = configs.pic3(n=args.n, width=args.width, height=args.height, dtype=dt)
            f2 = frames(ctx, s2, max(26, args.steps // 2), 3, log_prefix=f" {dt}")
            storage_images[dt] = f2["image_view0"]
            extras[dt] = dict(gsamples_per_s=round(f2["gsps"], 3), kernel_ms=round(f2["kernel_ms"], 4),
                              frame_ms_p50=round(float(np.median(f2["frame_ms"])), 4),
                              fps=round(max(26, args.steps // 2) / f2["elapsed"], 2), tile_shape=list(f2["shape"]),
                              samples_counted_by=f2["counted_by"])
        extras["iso"] = iso_frames(ctx, args.n, args.width, args.height)
        extras["encode_rgba8"] = encode(ctx, args.width, args.height)
        extras["jpeg"] = jpeg_frames(ctx, sc)
        extras["bricks8"] = bricks8(ctx, sc)
        extras["insitu"] = insitu_run(ctx, 128, args.width, args.height)
        extras["batch64"] = batch64(ctx, 10)
        extras["serving"] = serving(ctx, args.serve_seconds, 200.0)
        extras["serving_stress"] = serving(ctx, max(2.0, args.serve_seconds / 2), 2000.0)
        extras["serving_stress_5000"] = serving(ctx, max(2.0, args.serve_seconds / 4), 5000.0)
        extras["serving_unfrozen"] = serving(ctx, max(2.0, args.serve_seconds / 2), 200.0, freeze=False)
        extras["served_readback_ms"] = served_readback(ctx)
        out["extras"] = extras
    if not args.no_cpu_baseline:
        # every core this process may use, at most the host share of one GPU (16)
        threads = max(1, min(16, host_cpu()[1]))
        log(f"bench: CPU oracle baseline on 1 and {threads} threads")
        out["cpu_baseline"] = cpu_baseline(fr["scene_v0"], fr["image_view0"], fr["counts_view0"], threads,
                                           row_stride_all=args.cpu_row_stride, storage_images=storage_images)
        errs = out["cpu_baseline"]["storage_error_vs_oracle_of_fp32_fields"] or {}
        for dt, e in errs.items():
            if "extras" in out and dt in out["extras"]:
                out["extras"][dt]["error_vs_oracle_of_fp32_fields"] = e
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
