"""Batched renders: many sub-volumes in one persistent launch replayed as a hipGraph.

Each job rendered in a batch must equal the same job rendered alone, bit for
bit (the kernel body is shared; only the tile scheduling differs), across
graph replays with unrelated device work in between, and with the graph
switched off.  A sample of batch jobs is also checked against the oracle.
"""

import numpy as np
import pytest

import oracle
from parity import compare, log
from scenes import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0)
    yield c
    c.close()


def _setup(ctx, scenes_):
    import torch
    from paper_1611_09048_amd import device
    vols = [device.upload_volume(ctx, sc, vid) for vid, sc in enumerate(scenes_)]
    imgs = [device.new_image(sc) for sc in scenes_]
    cnts = [device.new_counts(sc) for sc in scenes_]
    jobs = [device.render_job(sc, vid, imgs[vid], cnts[vid]) for vid, sc in enumerate(scenes_)]
    torch.cuda.synchronize()
    return vols, imgs, cnts, jobs


def _mixed_scenes():
    out = configs.batch64(seed=4, n_jobs=10, edge=(20, 64), sizes=(48, 96, 130))
    out.append(configs.pic3(n=32, width=111, height=75))
    out.append(configs.plain_scalar(n=24, width=90, height=64))
    out.append(configs.pic3(n=24, width=40, height=33, dtype="bf16"))
    return out


def test_batch_equals_alone_bitwise(ctx):
    import torch
    from paper_1611_09048_amd import NO_GRAPH
    scenes_ = _mixed_scenes()
    log("batch of", len(scenes_), "jobs")
    vols, imgs, cnts, jobs = _setup(ctx, scenes_)
    alone = []
    for j, img, cnt in zip(jobs, imgs, cnts):
        ctx.render([j])
        torch.cuda.synchronize()
        alone.append((img.clone(), cnt.clone()))
    for mode, flags in (("graph", 0), ("direct", NO_GRAPH)):
        for rep in range(3):
            for img, cnt in zip(imgs, cnts):
                img.fill_(float("nan"))
                cnt.fill_(-7)
            # unrelated eager work and a host synchronisation between replays
            x = torch.randn(1 << 20, device="cuda")
            y = (x * 2.0).sum().item()
            assert np.isfinite(y)
            ctx.render(jobs, flags)
            torch.cuda.synchronize()
            for k, (img, cnt) in enumerate(zip(imgs, cnts)):
                assert torch.equal(img, alone[k][0]), (mode, rep, k)
                assert torch.equal(cnt, alone[k][1]), (mode, rep, k)
    del vols


def test_batch_of_maximum_size(ctx):
    """256 jobs (the most one call takes) on two volumes, each with its own camera and ragged
    image size, in one call: every job equals the same job rendered alone, bit for bit, with
    the graph and without; a sample of them also matches the oracle."""
    import torch
    from paper_1611_09048_amd import NO_GRAPH, binding, device
    assert binding.MAX_BATCH == 256
    bases = [configs.pic3(n=20, width=24, height=16), configs.plain_scalar(n=18, width=24, height=16)]
    vols = [device.upload_volume(ctx, sc, vid) for vid, sc in enumerate(bases)]
    views = configs.views26()
    scenes_, jobs, imgs, cnts = [], [], [], []
    for k in range(binding.MAX_BATCH):
        vid = k % 2
        base = bases[vid]
        sc = base.with_(camera=configs.orbit_camera(base.dims, views[k % 26], distance_factor=0.9 + 0.002 * k),
                        width=17 + k % 13, height=11 + k % 7)
        scenes_.append(sc)
        imgs.append(device.new_image(sc))
        cnts.append(device.new_counts(sc))
        jobs.append(device.render_job(sc, vid, imgs[-1], cnts[-1]))
    torch.cuda.synchronize()
    alone = []
    for j, img, cnt in zip(jobs, imgs, cnts):
        ctx.render([j])
        torch.cuda.synchronize()
        alone.append((img.clone(), cnt.clone()))
    assert sum(int((a[1] > 0).sum()) for a in alone) > 5000, "the jobs should see the volumes"
    for mode, flags in (("graph", 0), ("direct", NO_GRAPH)):
        for img, cnt in zip(imgs, cnts):
            img.fill_(float("nan"))
            cnt.fill_(-7)
        ctx.render(jobs, flags)
        torch.cuda.synchronize()
        for k, (img, cnt) in enumerate(zip(imgs, cnts)):
            assert torch.equal(img, alone[k][0]), (mode, k)
            assert torch.equal(cnt, alone[k][1]), (mode, k)
    for k in (0, 1, 77, 128, 254, 255):
        rec = oracle.render(scenes_[k])
        compare(imgs[k].cpu().numpy().reshape(-1, 4), cnts[k].cpu().numpy().reshape(-1), rec,
                label=f"batch of 256: job {k}")
    del vols


def test_batch_jobs_match_oracle(ctx):
    import torch
    scenes_ = _mixed_scenes()
    vols, imgs, cnts, jobs = _setup(ctx, scenes_)
    ctx.render(jobs)
    torch.cuda.synchronize()
    for k in (0, 3, 7, len(scenes_) - 3, len(scenes_) - 2, len(scenes_) - 1):
        sc = scenes_[k]
        rec = oracle.render(sc)
        compare(imgs[k].cpu().numpy().reshape(-1, 4), cnts[k].cpu().numpy().reshape(-1), rec,
                label=f"batch job {k} {sc.label}")
    del vols


def test_full_size_batch64_sampled(ctx):
    """The 64-job workload at its real sizes; every job compared with the oracle on sampled pixels."""
    import torch
    scenes_ = configs.batch64()
    vols, imgs, cnts, jobs = _setup(ctx, scenes_)
    ctx.render(jobs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    total = 0
    for k, sc in enumerate(scenes_):
        img = imgs[k].cpu().numpy()
        cnt = cnts[k].cpu().numpy()
        rows, cols = np.nonzero(img[..., 3] > 0)
        sel = rng.choice(rows.size, size=min(40, rows.size), replace=False) if rows.size else []
        px = np.array([(cols[i], rows[i]) for i in sel] + [(int(rng.integers(0, sc.width)),
                                                              int(rng.integers(0, sc.height))) for _ in range(10)],
                      dtype=np.int32)
        rec = oracle.render_pixels(sc, px)
        compare(img[px[:, 1], px[:, 0]], cnt[px[:, 1], px[:, 0]], rec, label=f"batch64[{k}]")
        total += int(rec["samples"].sum())
    assert total > 1e5
    del vols
