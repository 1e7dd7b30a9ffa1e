"""The pooled schedule (compacted rays handed to lane groups as they free up)
against the tiled schedule with the same lanes per ray: every ray is
composited by the same row-by-row arithmetic, so images, sample counts and
depths must agree bit for bit; and against the oracle.
"""

import numpy as np
import pytest

import oracle
from oracle.oracle import NO_TERMINATION
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
    for k in range(16):
        c.set_tile_shape(k, 8, 2, 1, 1, 0, 0)
    c.close()


def set_all(ctx, lanes, pooled, min_waves=0):
    for k in range(16):
        ctx.set_tile_shape(k, min(8, 64 // lanes), 2, 1, lanes, min_waves, pooled)


def render(ctx, sc, vid=0, flags=0, depth=False, **kw):
    import torch
    from paper_1611_09048_amd import device
    vol = device.upload_volume(ctx, sc, vid)
    img, cnt = device.new_image(sc), device.new_counts(sc)
    dep = torch.full((sc.height, sc.width), -1.0, device="cuda") if depth else None
    ctx.render([device.render_job(sc, vid, img, cnt, out_depth=dep.data_ptr() if depth else 0, **kw)], flags)
    torch.cuda.synchronize()
    out = (img.cpu().numpy(), cnt.cpu().numpy(), dep.cpu().numpy() if depth else None)
    del vol
    return out


def same(a, b, label):
    ok = all(np.array_equal(x, y) for x, y in zip(a, b) if x is not None)
    log(f"pooled vs tiled {label}: identical {ok}")
    assert ok, label


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_pooled_equals_tiled(ctx, lanes):
    from paper_1611_09048_amd import DERIVE, DIRECT
    scenes = [configs.pic3(n=48, width=200, height=150),
              configs.pic3(n=40, width=96, height=128, direction=(-0.2, -0.9, 0.3)),
              configs.plain_scalar(n=32, width=90, height=70)]
    for i, sc in enumerate(scenes):
        for flags in (DIRECT, DERIVE):
            for ert in (0.0, NO_TERMINATION):
                set_all(ctx, lanes, 0)
                a = render(ctx, sc, flags=flags, depth=True, ert_threshold=ert)
                set_all(ctx, lanes, 1)
                b = render(ctx, sc, flags=flags, depth=True, ert_threshold=ert)
                same(a, b, f"scene {i} lanes={lanes} flags={flags} ert={ert}")
    set_all(ctx, lanes, 1)
    for seed in range(12):
        sc = configs.random_small_scene(seed)
        img, cnt, _ = render(ctx, sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), oracle.render(sc), label=f"pooled random_small[{seed}] lanes={lanes}")


def test_pooled_full_parity_and_buffer_reuse(ctx):
    """A larger image after a smaller one (the ray list grows), repeated renders, min_waves variant."""
    set_all(ctx, 8, 1, 4)
    small = configs.pic3(n=48, width=64, height=48)
    big = configs.pic3(n=48, width=300, height=170)
    for sc in (small, big, small):
        img, cnt, _ = render(ctx, sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), oracle.render(sc, threads=8), label=f"pooled {sc.width}x{sc.height}")
        again, cnt2, _ = render(ctx, sc)
        assert np.array_equal(img, again) and np.array_equal(cnt, cnt2)


def test_pooled_bricks(ctx):
    """Bricks under the pooled schedule composite to the tiled result bit for bit."""
    import torch
    from paper_1611_09048_amd import device
    from test_gpu_bricks import render_bricks
    sc = configs.pic3(n=48, width=160, height=120)
    cuts = ([0, 17, 48], [0, 30, 48], [0, 9, 48])
    set_all(ctx, 4, 0)
    a, _ = render_bricks(ctx, sc, cuts)
    set_all(ctx, 4, 1)
    b, _ = render_bricks(ctx, sc, cuts)
    assert np.array_equal(a, b)
