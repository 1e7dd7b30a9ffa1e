"""Derived volumes: each active source's functor chain evaluated once per voxel
into an interleaved FP32 buffer that the ray loop then reads.  The loop would
compute the same values at every corner it visits, so a render through the
derived volume (ISAAC_DERIVE) must equal the direct render (ISAAC_DIRECT) bit
for bit, images and sample counts, in every mode and schedule.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from parity import compare, log
from scenes import configs, make_source, relayout

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0)
    yield c
    c.close()


def both(ctx, sc, vid=0, **overrides):
    from paper_1611_09048_amd import DERIVE, DIRECT, device
    a = device.render_scene(ctx, sc, volume_id=vid, flags=DIRECT, **overrides)
    b = device.render_scene(ctx, sc, volume_id=vid, flags=DERIVE, **overrides)
    return a, b


def assert_same(a, b, label):
    same_img = np.array_equal(a[0], b[0], equal_nan=True)
    same_cnt = a[1] is None or np.array_equal(a[1], b[1])
    log(f"derived vs direct {label}: max |diff| = {np.nanmax(np.abs(a[0] - b[0])):.3e}, counts equal {same_cnt}")
    assert same_img and same_cnt, label


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("interpolation", [1, 0])
def test_derived_equals_direct(ctx, dtype, interpolation):
    sc = configs.pic3(n=40, width=128, height=96, dtype=dtype).with_(interpolation=interpolation)
    a, b = both(ctx, sc)
    assert_same(a, b, f"pic3 {dtype} interp={interpolation}")
    if dtype == "f32" and interpolation == 1:
        compare(b[0].reshape(-1, 4), b[1].reshape(-1), oracle.render(sc, threads=8), label="derived vs oracle")


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_derived_every_schedule(ctx, lanes):
    from paper_1611_09048_amd import autotune
    sc = configs.pic3(n=40, width=128, height=96, direction=(-0.6, 0.3, 0.7))
    cls = autotune.size_class(sc.width, sc.height)
    old = ctx.get_tile_shape(cls)
    try:
        ctx.set_tile_shape(cls, 4 if lanes == 16 else 8, 2, 1, lanes, 0)
        a, b = both(ctx, sc)
        assert_same(a, b, f"lanes={lanes}")
    finally:
        ctx.set_tile_shape(cls, *old)


def test_derived_with_disabled_source_layouts_and_guardless(ctx):
    """A disabled middle source (components map around it), SoA and permuted
    layouts, a guard-less source and a non-persistent one."""
    from paper_1611_09048_amd import device
    base = configs.pic3(n=36, width=96, height=80)
    s0, s1, s2 = base.sources
    s1 = relayout(s1, layout="soa", order=(2, 0, 1))
    inner = s2.values[1:-1, 1:-1, 1:-1]
    s2g0 = make_source("B0", inner.astype(np.float32), guard=0, chain=s2.chain, weight=s2.weight, tf=s2.tf,
                       persistent=False)
    sc = base.with_(sources=[s0, s1, s2g0])
    a, b = both(ctx, sc, vid=3)
    assert_same(a, b, "soa/permuted + guard-less non-persistent")
    a, b = both(ctx, sc, vid=4, enabled=[True, False, True])
    assert_same(a, b, "middle source disabled")


def test_paired_layout_odd_extents(ctx):
    """Three-source derived volumes of a call whose jobs all run the three-source
    loop interleave (y, z) pairs: odd and unequal extents (padding pairs), nearest
    and trilinear.  Iso jobs and sources without guard layers (read by other
    loops) get the x-fastest layout; all equal the direct render."""
    base = configs.pic3(dims=(37, 35, 33), width=96, height=80, direction=(-0.7, 0.5, 0.5))
    for interp in (1, 0):
        a, b = both(ctx, base.with_(interpolation=interp), vid=20 + interp)
        assert_same(a, b, f"odd extents interp={interp}")
    iso = base.with_(mode="iso", sources=[dataclasses.replace(s, iso=v) for s, v in
                                          zip(base.sources, (1.0, 0.2, float("nan")))])
    a, b = both(ctx, iso, vid=22)
    assert_same(a, b, "odd extents iso")
    bare = [make_source(s.name, s.values[1:-1, 1:-1, 1:-1].astype(np.float32), guard=0, chain=s.chain,
                        weight=s.weight, tf=s.tf) for s in base.sources]
    a, b = both(ctx, base.with_(sources=bare), vid=23)
    assert_same(a, b, "odd extents, no guard layers")


def test_volume_and_iso_jobs_in_one_call(ctx):
    """A volume job and an iso job on one volume in the same call share one derived
    volume, which then keeps x-fastest order (the iso loop reads it); each image
    equals its direct render."""
    import torch
    from paper_1611_09048_amd import DERIVE, DIRECT, device
    sc = configs.pic3(n=40, width=112, height=80, direction=(0.3, -0.8, 0.5))
    iso = sc.with_(mode="iso", sources=[dataclasses.replace(s, iso=v) for s, v in
                                        zip(sc.sources, (1.0, 0.2, float("nan")))])
    vol = device.upload_volume(ctx, sc, 24)
    out = {}
    for flags in (DIRECT, DERIVE):
        imgs = [device.new_image(sc), device.new_image(iso)]
        ctx.render([device.render_job(sc, 24, imgs[0]), device.render_job(iso, 24, imgs[1])], flags)
        torch.cuda.synchronize()
        out[flags] = [im.cpu().numpy() for im in imgs]
    for k, label in enumerate(("volume", "iso")):
        assert np.array_equal(out[DIRECT][k], out[DERIVE][k], equal_nan=True), label
    log("volume + iso in one call: derived equals direct")
    del vol


def test_derived_iso_mode(ctx):
    sc = configs.pic3(n=40, width=128, height=96)
    sc = sc.with_(mode="iso", sources=[dataclasses.replace(s, iso=v) for s, v in
                                       zip(sc.sources, (1.0, 0.2, float("nan")))])
    a, b = both(ctx, sc, vid=5)
    assert_same(a, b, "iso")


def test_derived_batch_of_views(ctx):
    """Several jobs on one volume with different enabled sets and clip planes share
    one derived volume; voxels clipped away for every job are not derived."""
    import torch
    from paper_1611_09048_amd import DERIVE, DIRECT, device
    sc = configs.pic3(n=40, width=112, height=80)
    vol = device.upload_volume(ctx, sc, 6)
    views = [configs.D0, (0.2, -0.9, 0.4), (-0.7, -0.1, -0.7)]
    enabled = [None, [True, False, True], [False, True, True]]
    rng = np.random.default_rng(21)
    clips = [[configs.random_clip_plane(rng, sc.dims) for _ in range(k)] for k in (1, 3, 2)]
    out = {}
    for flags in (DIRECT, DERIVE):
        imgs = [device.new_image(sc) for _ in views]
        jobs = [device.render_job(sc.with_(camera=configs.orbit_camera(sc.dims, v), clip=c), 6, im, enabled=e)
                for v, im, e, c in zip(views, imgs, enabled, clips)]
        for _ in range(3):                      # graph replays included
            ctx.render(jobs, flags)
        torch.cuda.synchronize()
        out[flags] = [im.cpu().numpy() for im in imgs]
    for k in range(len(views)):
        assert np.array_equal(out[DIRECT][k], out[DERIVE][k]), k
    del vol


def test_derived_skips_clipped_voxels_only(ctx):
    """Clip planes cutting most of the volume away, in volume and iso mode, nearest
    and trilinear: the skipped voxels are never read (derived equals direct)."""
    base = configs.pic3(n=40, width=128, height=96, direction=(0.5, 0.6, -0.6))
    c = np.array(base.dims, dtype=np.float64) / 2
    for k, (normal, off) in enumerate((((1.0, 0.2, 0.1), 6.0), ((-0.3, 1.0, 0.4), -3.0), ((0.0, 0.0, 1.0), 12.0))):
        nrm = np.array(normal) / np.linalg.norm(normal)
        plane = (float(nrm[0]), float(nrm[1]), float(nrm[2]), float(-(nrm @ c) - off))
        sc = base.with_(clip=[plane], interpolation=k % 2)
        a, b = both(ctx, sc, vid=7)
        assert_same(a, b, f"heavy clip {k}")
    iso = base.with_(clip=[plane], mode="iso",
                     sources=[dataclasses.replace(s, iso=v) for s, v in zip(base.sources, (1.0, 0.2, float("nan")))])
    a, b = both(ctx, iso, vid=8)
    assert_same(a, b, "heavy clip iso")


def render_into(ctx, sc, vid, flags=0, **overrides):
    import torch
    from paper_1611_09048_amd import device
    img, cnt = device.new_image(sc), device.new_counts(sc)
    ctx.render([device.render_job(sc, vid, img, cnt, **overrides)], flags)
    torch.cuda.synchronize()
    return img.cpu().numpy(), cnt.cpu().numpy()


def test_frozen_volume_equals_direct(ctx):
    """isaac_freeze_volume: one derive of every source, then renders with other clip planes,
    a source disabled, the iso mode and served requests all equal the direct renders."""
    import torch
    from paper_1611_09048_amd import DIRECT, device
    sc = configs.pic3(n=40, width=128, height=96, direction=(0.5, -0.4, 0.7))
    vol = device.upload_volume(ctx, sc, 11)
    ctx.freeze_volume(11)
    ctx.freeze_volume(11)                               # already frozen: no-op
    cases = [("as scene", sc, {}),
             ("no clip", sc.with_(clip=[]), {}),
             ("other view", sc.with_(camera=configs.orbit_camera(sc.dims, (-0.3, 0.8, -0.5))), {}),
             ("source 1 off", sc, dict(enabled=[1, 0, 1])),
             ("nearest", sc.with_(interpolation=0), {})]
    for label, s, kw in cases:
        a = render_into(ctx, s, 11, DIRECT, **kw)
        b = render_into(ctx, s, 11, 0, **kw)
        assert_same(a, b, f"frozen {label}")
    iso = sc.with_(mode="iso", sources=[dataclasses.replace(x, iso=v) for x, v in
                                        zip(sc.sources, (1.0, 0.2, float("nan")))])
    assert_same(render_into(ctx, iso, 11, DIRECT), render_into(ctx, iso, 11, 0), "frozen iso")
    # a served request reads the frozen values too
    t = ctx.submit(device.render_job(sc, 11, device.new_image(sc)))
    served = ctx.read_image(t, np.zeros((sc.height, sc.width, 4), dtype=np.float32))
    ctx.release(t)
    direct = render_into(ctx, sc, 11, DIRECT)[0]
    assert np.array_equal(served, direct)
    # redefinition thaws: new data is read
    sc2 = configs.pic3(n=40, width=128, height=96, seed=99, direction=(0.5, -0.4, 0.7))
    vol2 = device.upload_volume(ctx, sc2, 11)
    assert_same(render_into(ctx, sc2, 11, DIRECT), render_into(ctx, sc2, 11, 0), "thawed after redefinition")
    img, cnt = render_into(ctx, sc2, 11, 0)
    compare(img.reshape(-1, 4), cnt.reshape(-1), oracle.render(sc2, threads=8), label="thawed vs oracle")
    del vol, vol2
    torch.cuda.synchronize()


def test_freeze_rejections_and_plain_volume(ctx):
    from paper_1611_09048_amd import DIRECT, binding, device
    with pytest.raises(binding.IsaacError) as e:
        ctx.freeze_volume(200)                          # never defined
    assert e.value.code == -6
    base = configs.pic3(n=24, width=48, height=40)
    s0, s1, s2 = base.sources
    sc = base.with_(sources=[s0, s1, dataclasses.replace(s2, persistent=False)])
    vol = device.upload_volume(ctx, sc, 12)
    with pytest.raises(binding.IsaacError) as e:
        ctx.freeze_volume(12)
    assert e.value.code == -1
    plain = configs.plain_scalar(n=32, width=64, height=48)
    vol2 = device.upload_volume(ctx, plain, 13)
    ctx.freeze_volume(13)                               # plain FP32 scalar: read directly, nothing to freeze
    assert_same(render_into(ctx, plain, 13, DIRECT), render_into(ctx, plain, 13, 0), "plain frozen")
    del vol, vol2
