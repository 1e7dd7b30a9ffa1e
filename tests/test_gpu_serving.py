"""Serving: requests batched on arrival give the same image as each request rendered alone."""

import time

import numpy as np
import pytest

import oracle
from parity import compare, log, pixel_list
from scenes import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0, mem_budget=64 << 20, max_inflight=24)
    yield c
    c.close()


def test_served_images_equal_alone_renders(ctx):
    import torch
    from paper_1611_09048_amd import device, serve
    dims = (48, 40, 36)
    vol_scene = configs.pic3(dims=dims, width=8, height=8)
    vol = device.upload_volume(ctx, vol_scene, 7)
    ex = serve.DeviceExecutor(ctx, vol, dims)
    images = {}
    jobs = {}

    def on_done(rec, ticket):
        h, w = rec.height, rec.width
        images[rec.rid] = ctx.read_image(ticket, np.empty((h, w, 4), dtype=np.float32))

    srv = serve.Server(ex, time.perf_counter, max_batch=6, max_batches_in_flight=3, on_done=on_done)
    reqs = configs.serving_requests(21, dims, n_clients=3, rate_per_client=400.0, duration=0.12,
                                    base_tfs=[s.tf for s in vol_scene.sources])
    reqs = [r.__class__(**{**r.__dict__, "width": (64, 97, 130)[i % 3], "height": (64, 55, 71)[i % 3]})
            for i, r in enumerate(reqs)]

    def make_job(i, r):
        j = serve.job_from_request(i, r)
        jobs[i] = j
        return j

    dur = serve.run(srv, reqs, time.perf_counter, make_job=make_job)
    s = srv.summary(dur)
    log("serving test summary", s)
    assert s["completed"] == len(reqs) and s["failed"] == 0
    assert s["batches"] < len(reqs)                 # requests were batched
    used, budget, inflight = ctx.serving_usage()
    assert inflight == 0 and used == 0
    # each request alone, through isaac_render, with the same descriptor
    for rid, j in jobs.items():
        desc, _ = ex.desc(j)
        out = torch.full((j.height, j.width, 4), float("nan"), dtype=torch.float32, device="cuda")
        desc.out_rgba = out.data_ptr()
        ctx.render([desc])
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), images[rid]), rid
    # and a few against the oracle
    for rid in list(jobs)[:3]:
        j = jobs[rid]
        eye, center, up = ex.camera(j.direction)
        from scenes.layout import Camera
        srcs = [s.__class__(**{**s.__dict__, "tf": j.tfs[k]}) for k, s in enumerate(vol_scene.sources)]
        sc = vol_scene.with_(sources=srcs, camera=Camera(eye=eye, center=center, up=up), width=j.width,
                             height=j.height, clip=j.clip)
        compare(images[rid].reshape(-1, 4), None, oracle.render(sc), label=f"served request {rid}")
    del vol


def test_admission_refused_when_budget_is_full(ctx):
    from paper_1611_09048_amd import device
    sc = configs.pic3(n=16, width=1024, height=1024)
    vol = device.upload_volume(ctx, sc, 8)
    job = device.render_job(sc, 8, device.new_image(sc))
    tickets = []
    while True:
        t = ctx.submit(job)
        if t is None:
            break
        tickets.append(t)
        assert len(tickets) <= 4
    assert len(tickets) == 4               # 64 MiB budget / 16 MiB images
    for t in tickets:
        ctx.release(t)
    assert ctx.serving_usage()[0] == 0
    t = ctx.submit(job)
    assert t is not None
    ctx.release(t)
    del vol


def test_budget_runs_merge_after_release_in_any_order(ctx):
    """Served images are carved from one block of the budget: images of three sizes
    released out of order leave one free run again, so an image of the whole budget
    (64 MiB) is admitted afterwards; an image larger than the budget never is."""
    from paper_1611_09048_amd import device
    sc = configs.pic3(n=16, width=64, height=64)
    vol = device.upload_volume(ctx, sc, 9)
    out = device.new_image(sc)
    sizes = [(1024, 1024), (512, 512), (2048, 1024), (512, 512)]
    tickets = [ctx.submit(device.render_job(sc.with_(width=w, height=h), 9, out)) for w, h in sizes]
    assert all(t is not None for t in tickets)
    for k in (1, 0, 3, 2):
        ctx.release(tickets[k])
    assert ctx.serving_usage()[0] == 0
    whole = ctx.submit(device.render_job(sc.with_(width=2048, height=2048), 9, out))
    assert whole is not None                       # 2048 x 2048 x 16 B = the 64 MiB budget
    assert ctx.submit(device.render_job(sc, 9, out)) is None       # nothing left beside it
    ctx.release(whole)
    assert ctx.submit(device.render_job(sc.with_(width=4096, height=2048), 9, out)) is None
    assert ctx.serving_usage()[0] == 0
    del vol


def test_served_full_size_sampled():
    """The serving workload at its real sizes: the 512x512x256 three-source volume,
    frozen as the benchmark serves it, one request at each resolution (512x512,
    1280x720, 1920x1080) through the continuous-batching loop; every served image
    compared with the oracle on sampled pixels."""
    from paper_1611_09048_amd import Context, device, serve
    from scenes.layout import Camera
    c = Context(device=0)
    try:
        dims = (512, 512, 256)
        vol_scene = configs.pic3(dims=dims, width=16, height=16)
        vol = device.upload_volume(c, vol_scene, 200)
        c.freeze_volume(200)
        ex = serve.DeviceExecutor(c, vol, dims)
        images, jobs = {}, {}

        def on_done(rec, ticket):
            images[rec.rid] = c.read_image(ticket, np.empty((rec.height, rec.width, 4), dtype=np.float32))

        def make_job(i, r):
            jobs[i] = serve.job_from_request(i, r)
            return jobs[i]

        srv = serve.Server(ex, time.perf_counter, max_batch=16, max_batches_in_flight=3, on_done=on_done)
        reqs = configs.serving_requests(11, dims, n_clients=4, rate_per_client=200.0, duration=0.05,
                                        base_tfs=[s.tf for s in vol_scene.sources])
        sizes = [(512, 512), (1280, 720), (1920, 1080)]
        reqs = [r.__class__(**{**r.__dict__, "width": sizes[i][0], "height": sizes[i][1]})
                for i, r in enumerate(reqs[:3])]
        assert len(reqs) == 3
        dur = serve.run(srv, reqs, time.perf_counter, make_job=make_job)
        summary = srv.summary(dur)
        log("full-size serving summary", summary)
        assert summary["completed"] == 3 and summary["failed"] == 0
        rng = np.random.default_rng(12)
        for rid, j in jobs.items():
            eye, center, up = ex.camera(j.direction)
            srcs = [s.__class__(**{**s.__dict__, "tf": j.tfs[k]}) for k, s in enumerate(vol_scene.sources)]
            sc = vol_scene.with_(sources=srcs, camera=Camera(eye=eye, center=center, up=up), width=j.width,
                                 height=j.height, clip=j.clip)
            img = images[rid]
            assert np.isfinite(img).all()
            px = pixel_list(j.height, j.width, 300, rng, hit_mask=img[..., 3] > 0, n_hit=700)
            rec = oracle.render_pixels(sc, px)
            compare(img[px[:, 1], px[:, 0]], None, rec, label=f"served {j.width}x{j.height} request {rid}")
        del vol
    finally:
        c.close()
