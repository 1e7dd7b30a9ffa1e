"""isaac_render_noalloc (the render entry point for callers that cannot
allocate) against isaac_render, through the C ABI: the same images and sample
counts bit for bit on two calls in a row (the second smaller), on a batch, on
a frozen volume and on a non-persistent source; sizes beyond its static
scratch and flags it does not take are refused before anything runs."""

import ctypes

import numpy as np
import pytest

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


def _pair(ctx, scene, vid, flags=0, **overrides):
    """(image, counts) from isaac_render and from isaac_render_noalloc, same job."""
    import torch
    from paper_1611_09048_amd import device
    out = []
    for noalloc in (False, True):
        img, cnt = device.new_image(scene), device.new_counts(scene)
        job = device.render_job(scene, vid, img, cnt, **overrides)
        log("render", "noalloc" if noalloc else "render", scene.dims, scene.width, "x", scene.height)
        (ctx.render_noalloc if noalloc else ctx.render)([job], flags)
        torch.cuda.synchronize()
        out.append((img.cpu().numpy(), cnt.cpu().numpy()))
    return out


def test_noalloc_equals_render_on_two_calls_in_a_row(ctx):
    import oracle
    from paper_1611_09048_amd import device
    big = configs.pic3(n=64, width=320, height=240)
    small = configs.pic3(n=32, width=96, height=64, direction=(0.2, -1.0, 0.4))
    vb = device.upload_volume(ctx, big, 60)
    vs = device.upload_volume(ctx, small, 61)
    (ri, rc), (ni, nc) = _pair(ctx, big, 60)
    assert np.array_equal(ri, ni, equal_nan=True) and np.array_equal(rc, nc)
    assert (nc > 0).sum() > 1000
    compare(ni.reshape(-1, 4), nc.reshape(-1), oracle.render(big), label="noalloc pic3 64^3 320x240")
    # second call, smaller: the scratch holds the first call's records, every one rewritten or unread
    (ri2, rc2), (ni2, nc2) = _pair(ctx, small, 61)
    assert np.array_equal(ri2, ni2, equal_nan=True) and np.array_equal(rc2, nc2)
    compare(ni2.reshape(-1, 4), nc2.reshape(-1), oracle.render(small), label="noalloc pic3 32^3 96x64")
    del vb, vs


def test_noalloc_batch_frozen_and_nonpersistent(ctx):
    import torch
    from paper_1611_09048_amd import device
    a = configs.pic3(n=48, width=200, height=150)
    b = configs.pic3(n=40, width=128, height=128, direction=(-0.3, 0.9, 0.2))
    va, vb = device.upload_volume(ctx, a, 62), device.upload_volume(ctx, b, 63)
    imgs = {}
    for noalloc in (False, True):
        ia, ib = device.new_image(a), device.new_image(b)
        jobs = [device.render_job(a, 62, ia), device.render_job(b, 63, ib)]
        (ctx.render_noalloc if noalloc else ctx.render)(jobs)
        torch.cuda.synchronize()
        imgs[noalloc] = (ia.cpu().numpy(), ib.cpu().numpy())
    for x, y in zip(imgs[False], imgs[True]):
        assert np.array_equal(x, y, equal_nan=True)
    # a frozen volume: the no-alloc call reads the frozen derived values
    ctx.freeze_volume(63)
    (ri, rc), (ni, nc) = _pair(ctx, b, 63)
    assert np.array_equal(ri, ni, equal_nan=True) and np.array_equal(rc, nc)
    assert np.array_equal(ni, imgs[True][1], equal_nan=True)
    del va, vb
    # a non-persistent source: copied into the buffer isaac_set_sources allocated
    import dataclasses
    c = configs.pic3(n=32, width=96, height=96)
    c = c.with_(sources=[dataclasses.replace(s, persistent=(k != 1)) for k, s in enumerate(c.sources)])
    vc = device.upload_volume(ctx, c, 64)
    (ri, rc), (ni, nc) = _pair(ctx, c, 64)
    assert np.array_equal(ri, ni, equal_nan=True) and np.array_equal(rc, nc)
    del vc


def test_noalloc_refuses_what_does_not_fit(ctx):
    import torch
    from paper_1611_09048_amd import ASYNC, TIMING, DERIVE, binding, device
    sc = configs.pic3(n=32, width=64, height=64)
    v = device.upload_volume(ctx, sc, 65)
    img = device.new_image(sc)
    job = device.render_job(sc, 65, img)
    for flags in (TIMING, DERIVE, ASYNC | TIMING):
        with pytest.raises(binding.IsaacError) as e:
            ctx.render_noalloc([job], flags)
        assert e.value.code == -1 and "takes" in str(e.value)
    # a 2048x2048 view of a volume that fills the screen: 4M rectangle pixels, above the scratch
    near = sc.with_(width=2048, height=2048,
                    camera=configs.orbit_camera(sc.dims, (0.0, 0.0, 1.0), distance_factor=0.6))
    big = torch.full((2048, 2048, 4), 7.0, device="cuda")
    with pytest.raises(binding.IsaacError) as e:
        ctx.render_noalloc([device.render_job(near, 65, big)])
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((big == 7.0).all())                 # nothing ran
    lib = binding.load()
    assert ctypes.sizeof(ctypes.c_char) == 1 and hasattr(lib, "isaac_render_noalloc")
    del v
