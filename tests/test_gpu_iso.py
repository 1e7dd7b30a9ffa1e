"""Iso-surface mode on the GPU against the oracle, through the C ABI.

The surface is the first crossing of a source's interpolated chain output
through its iso value between consecutive scan points, placed linearly and
shaded by a headlight with the central-difference gradient.  Pixels whose
crossing decision lies within the oracle's iso margin are unconstrained;
every other pixel matches within the parity tolerance, and its sample count
exactly.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from parity import compare, log
from scenes import Camera, Scene, configs, make_source

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0)
    yield c
    c.close()


def chain_quantile(src, q, rng, n=400):
    """A quantile of the source's chain output over random stored voxels, rounded to FP32."""
    v = src.values.reshape(-1, src.f_dim)
    vals = [oracle.chain_eval(src.chain, src.f_dim, v[i])[0] for i in rng.integers(0, v.shape[0], size=n)]
    return float(np.float32(np.quantile(vals, q)))


def iso_scene(n=48, width=160, height=120, isos=(0.6, 0.5, None), direction=configs.D0, interpolation=1,
              n_clip=2):
    sc = configs.pic3(n=n, width=width, height=height, direction=direction, n_clip=n_clip)
    rng = np.random.default_rng(11)
    srcs = []
    for s, q in zip(sc.sources, isos):
        srcs.append(dataclasses.replace(s, iso=float("nan") if q is None else chain_quantile(s, q, rng)))
    return sc.with_(sources=srcs, mode="iso", interpolation=interpolation)


def render(ctx, sc, vid=0):
    from paper_1611_09048_amd import device
    img, cnt = device.render_scene(ctx, sc, volume_id=vid)
    return img.reshape(-1, 4), cnt.reshape(-1)


@pytest.mark.parametrize("interpolation", [1, 0])
@pytest.mark.parametrize("direction", [configs.D0, (-0.4, -0.2, 0.9)])
def test_iso_matches_oracle(ctx, interpolation, direction):
    sc = iso_scene(direction=direction, interpolation=interpolation)
    img, cnt = render(ctx, sc)
    rec = oracle.render(sc, threads=8)
    st = compare(img, cnt, rec, label=f"iso interp={interpolation} dir={direction}")
    hits = rec["rgba"][:, 3] == 1.0
    assert hits.sum() > 300, "the scene should show a surface"
    assert np.all((img[:, 3] == 0.0) | (img[:, 3] == 1.0))
    # a pixel whose crossing decision lies within its margin is unconstrained: few of the surface
    assert st["unconstrained_pixels"] <= 0.05 * hits.sum(), (st["unconstrained_pixels"], int(hits.sum()))


def test_iso_two_surfaces_and_clip(ctx):
    """Two sources with surfaces (the first crossing of either wins) and no clip planes."""
    sc = iso_scene(isos=(0.7, 0.4, 0.6), n_clip=0, direction=(0.3, -0.8, 0.5))
    img, cnt = render(ctx, sc)
    compare(img, cnt, oracle.render(sc, threads=8), label="iso three sources")


def test_iso_bilinear_closed_form(ctx):
    """v = a x + c x z + b: exact crossings and normals (the oracle's closed-form pin, on the GPU)."""
    a_, c_, b_ = 0.0625, 0.015625, 0.125
    xs = np.arange(-1, 17) + 0.5
    zs = np.arange(-1, 7) + 0.5
    v = (a_ * xs[None, None, :] + c_ * xs[None, None, :] * zs[:, None, None] + b_) * np.ones((8, 8, 18))
    iso = float(np.float32(b_ + (a_ + 3.0 * c_) * 5.1))
    src = make_source("bilinear", v[..., None], guard=1, iso=iso,
                      tf=[(0.0, 0.9, 0.5, 0.1, 0.2), (1.0, 0.1, 0.5, 0.9, 0.7)])
    for sign in (1.0, -1.0):
        cam = Camera(eye=(8.0 - sign * 20.0, 3.0, 3.0), center=(8.0, 3.0, 3.0), up=(0.0, 0.0, 1.0),
                     projection="orthographic", ortho_height=3.0)
        sc = Scene(dims=(16, 6, 6), sources=[src], camera=cam, width=33, height=17, step=0.5, interpolation=1,
                   ert_threshold=1.0, mode="iso")
        img, cnt = render(ctx, sc)
        rec = oracle.render(sc)
        st = compare(img, cnt, rec, label=f"iso bilinear sign={sign}")
        assert st["unconstrained_pixels"] <= 0.05 * img.shape[0]
        assert np.all(img[:, 3] == 1.0)


def test_iso_without_surfaces_and_mixed_batch(ctx):
    """No iso value: nothing drawn, every kept point counted.  An iso job batched with
    a volume job renders exactly as each does alone."""
    import torch
    from paper_1611_09048_amd import device
    sc_iso = iso_scene(n=32, width=96, height=64)
    none = sc_iso.with_(sources=[dataclasses.replace(s, iso=float("nan")) for s in sc_iso.sources])
    img, cnt = render(ctx, none)
    rec = oracle.render(none, threads=8)
    assert np.all(img == 0.0)
    compare(img, cnt, rec, label="iso without surfaces")
    sc_vol = sc_iso.with_(mode="volume")
    alone_iso, _ = render(ctx, sc_iso)
    alone_vol, _ = render(ctx, sc_vol)
    vol = device.upload_volume(ctx, sc_iso, 5)
    a, b = device.new_image(sc_iso), device.new_image(sc_vol)
    ctx.render([device.render_job(sc_iso, 5, a), device.render_job(sc_vol, 5, b)])
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy().reshape(-1, 4), alone_iso)
    assert np.array_equal(b.cpu().numpy().reshape(-1, 4), alone_vol)
    del vol


def test_iso_rejects_bricks(ctx):
    from paper_1611_09048_amd import binding, device
    sc = iso_scene(n=16, width=8, height=8)
    vol = device.upload_volume(ctx, sc, 7)
    img = device.new_image(sc)
    with pytest.raises(binding.IsaacError) as e:
        ctx.render([device.render_job(sc, 7, img, brick_origin=(0, 0, 0), global_dims=sc.dims)])
    assert e.value.code == -1
    with pytest.raises(binding.IsaacError):
        ctx.render([device.render_job(sc, 7, img, mode=2)])
    del vol


def _with_shape(ctx, sc, shape):
    """Render sc with `shape` as its size class's tile shape; restores the previous one."""
    from paper_1611_09048_amd import autotune
    cls = autotune.size_class(sc.width, sc.height)
    old = ctx.get_tile_shape(cls)
    try:
        ctx.set_tile_shape(cls, *shape)
        return render(ctx, sc)
    finally:
        ctx.set_tile_shape(cls, *old)


@pytest.mark.parametrize("interpolation", [1, 0])
@pytest.mark.parametrize("isos", [(0.6, 0.5, 0.55), (None, 0.45, None), (0.2, None, 0.9)])
def test_iso_lanes_equal_one_lane(ctx, interpolation, isos):
    """Several lanes per ray (8: the size class asks for 16) find the same crossing, source,
    fraction and count as one lane per ray, bit for bit: every lane tests its own pair of
    consecutive scan points and the first one wins.  Two clip planes, ragged image."""
    sc = iso_scene(n=40, width=131, height=97, isos=isos, direction=(-0.4, -0.2, 0.9),
                   interpolation=interpolation)
    one_img, one_cnt = _with_shape(ctx, sc, (8, 2, 1, 1, 0, 0))
    lanes_img, lanes_cnt = _with_shape(ctx, sc, (4, 1, 1, 16, 0, 0))
    assert np.array_equal(one_img, lanes_img) and np.array_equal(one_cnt, lanes_cnt)
    assert (lanes_img[:, 3] == 1.0).sum() > 100 or isos == (None, None, None)


def test_iso_full_size_sampled(ctx):
    """The iso-surface form of the 256^3 1080p benchmark scene (density surface at 1.0, |E| at
    0.2, B without a surface) in its launch configuration (the benchmark's tuned tile shape, so
    8 lanes per ray); sampled pixels, hit pixels included."""
    import os
    from paper_1611_09048_amd import autotune
    from parity import pixel_list
    sc = configs.pic3()
    sc = sc.with_(mode="iso", sources=[dataclasses.replace(s, iso=v) for s, v in
                                       zip(sc.sources, (1.0, 0.2, float("nan")))])
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = autotune.load_cache(os.path.join(root, "paper_1611_09048_amd", "tuned_gfx950.json"))
    shape = cache[autotune.cache_key("gfx950", str(autotune.size_class(sc.width, sc.height)), "pic3:f32")]
    img, cnt = _with_shape(ctx, sc, shape)
    img = img.reshape(sc.height, sc.width, 4)
    cnt = cnt.reshape(sc.height, sc.width)
    rng = np.random.default_rng(5)
    px = pixel_list(sc.height, sc.width, 1000, rng, extra_rows=(540,), extra_cols=(960,),
                    hit_mask=img[..., 3] > 0, n_hit=2000)
    rec = oracle.render_pixels(sc, px)
    st = compare(img[px[:, 1], px[:, 0]], cnt[px[:, 1], px[:, 0]], rec, label="iso pic3 256^3 1080p sampled")
    hits = rec["rgba"][:, 3] == 1.0
    assert hits.sum() > 500, "the sample should contain surface pixels"
    # a pixel whose crossing decision lies within its margin is unconstrained: few of the surface
    assert st["unconstrained_pixels"] <= 0.05 * hits.sum(), (st["unconstrained_pixels"], int(hits.sum()))
    assert np.all((img[..., 3] == 0.0) | (img[..., 3] == 1.0))
