"""Sort-last rendering on one GPU: bricks on the global step grid, then over-compositing.

A volume is cut into bricks, each stored with one guard layer copied from the
global field (as neighbouring ranks would provide them, Sec. 3.1); each brick
renders only the scan points inside its own box and writes the depth of its
first scan point; isaac_composite orders the partial images per pixel and
combines them front to back.  Without early termination the result must
equal the whole-volume render up to FP32 rounding of the compositing order,
and the oracle's whole-volume image within the parity tolerance.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from oracle.oracle import NO_TERMINATION
from parity import compare, log
from scenes import configs, make_source

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0)
    yield c
    c.close()


def brick_sources(scene, lo, hi):
    """The scene's sources restricted to cells [lo, hi) plus one guard layer from the global field."""
    out = []
    for s in scene.sources:
        g = s.guard
        assert g == 1
        v = s.values[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2]   # global index i -> array i + 1
        b = make_source(s.name, v.astype(np.float32) if s.dtype == "f32" else v, dtype=s.dtype, guard=1,
                        chain=s.chain, weight=s.weight, tf=s.tf)
        assert np.array_equal(b.values, v)
        out.append(b)
    return out


def render_bricks(ctx, scene, cuts, ert=NO_TERMINATION):
    import torch
    from paper_1611_09048_amd import device
    dims = scene.dims
    layers, depths, vols = [], [], []
    vid = 20
    for i in range(len(cuts[0]) - 1):
        for j in range(len(cuts[1]) - 1):
            for k in range(len(cuts[2]) - 1):
                lo = (cuts[0][i], cuts[1][j], cuts[2][k])
                hi = (cuts[0][i + 1], cuts[1][j + 1], cuts[2][k + 1])
                bdims = tuple(h - l for l, h in zip(lo, hi))
                bs = scene.with_(dims=bdims, sources=brick_sources(scene, lo, hi))
                vols.append(device.upload_volume(ctx, bs, vid))
                img = device.new_image(scene)
                dep = torch.full((scene.height, scene.width), float("nan"), device="cuda")
                ctx.render([device.render_job(scene, vid, img, brick_origin=lo, global_dims=dims,
                                              out_depth=dep.data_ptr(), ert_threshold=ert)])
                layers.append(img)
                depths.append(dep)
                vid += 1
    out = device.new_image(scene)
    ctx.composite([l.data_ptr() for l in layers], [d.data_ptr() for d in depths], scene.width, scene.height,
                  out.data_ptr())
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    del vols
    return res, len(layers)


@pytest.mark.parametrize("cuts_kind", ["halves", "uneven"])
@pytest.mark.parametrize("direction", [configs.D0, (-0.3, 0.9, -0.5)])
def test_bricks_composite_to_the_whole_image(ctx, cuts_kind, direction):
    from paper_1611_09048_amd import device
    sc = configs.pic3(n=48, width=160, height=120, direction=direction)
    n = 48
    cuts = ([0, 24, 48],) * 3 if cuts_kind == "halves" else ([0, 17, 48], [0, 30, 41, 48], [0, 9, 48])
    whole, _ = device.render_scene(ctx, sc, ert_threshold=NO_TERMINATION, count=False)
    comp, nl = render_bricks(ctx, sc, cuts)
    log(f"bricks {cuts_kind} ({nl} layers) dir={direction}: max |composite - whole| = {np.abs(comp - whole).max():.3e}")
    assert np.isfinite(comp).all()
    assert np.abs(comp - whole).max() <= 1e-6
    rec = oracle.render(sc, ert_threshold=NO_TERMINATION)
    compare(comp.reshape(-1, 4), None, rec, label=f"composite of {nl} bricks vs oracle")


def test_brick_depth_and_single_layer(ctx):
    """A brick equal to the whole volume reproduces the whole render bit for bit; depth is +inf off the box."""
    import torch
    from paper_1611_09048_amd import device
    sc = configs.pic3(n=32, width=90, height=70)
    whole, cnt = device.render_scene(ctx, sc, ert_threshold=NO_TERMINATION)
    vol = device.upload_volume(ctx, sc, 60)
    img = device.new_image(sc)
    dep = torch.zeros((sc.height, sc.width), device="cuda")
    ctx.render([device.render_job(sc, 60, img, brick_origin=(0, 0, 0), global_dims=sc.dims,
                                  out_depth=dep.data_ptr(), ert_threshold=NO_TERMINATION)])
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy(), whole)
    d = dep.cpu().numpy()
    assert np.array_equal(np.isfinite(d), cnt > 0)
    assert (cnt > 0).any() and (cnt == 0).any()
    del vol


def test_bricks_full_size(ctx):
    """The benchmark volume (256^3, 1920x1080) cut into 8 bricks of 128^3, as 8 ranks would hold
    it: the composite equals the whole-volume render to FP32 compositing order, and sampled
    pixels match the oracle."""
    from paper_1611_09048_amd import device
    from parity import pixel_list
    sc = configs.pic3()
    whole, _ = device.render_scene(ctx, sc, ert_threshold=NO_TERMINATION, count=False)
    comp, nl = render_bricks(ctx, sc, ([0, 128, 256],) * 3)
    diff = np.abs(comp - whole).max()
    log(f"bricks 256^3 1080p ({nl} layers): max |composite - whole| = {diff:.3e}")
    assert nl == 8 and np.isfinite(comp).all()
    assert diff <= 1e-5
    rng = np.random.default_rng(8)
    px = pixel_list(sc.height, sc.width, 500, rng, hit_mask=whole[..., 3] > 0, n_hit=1500)
    rec = oracle.render_pixels(sc, px, ert_threshold=NO_TERMINATION)
    compare(comp[px[:, 1], px[:, 0]], None, rec, label="8-brick composite 1080p vs oracle (sampled)")


@pytest.mark.parametrize("n_layers", [1, 3, 8, 16])
def test_composite_order_ties_and_uncovered_layers(ctx, n_layers):
    """isaac_composite on synthetic layers against its definition: per pixel the layers
    with a finite depth in depth order (ties in layer order), combined front to back;
    a layer whose depth is +inf is not read there (its colour may be anything), and a
    pixel no layer covers is transparent black, exactly.  Ragged size (3 partial waves)."""
    import torch
    rng = np.random.default_rng(50 + n_layers)
    h, w = 37, 61
    depth = rng.choice([1.0, 2.0, 2.5, 3.0, 7.0], size=(n_layers, h, w)).astype(np.float32)   # ties
    depth[rng.random((n_layers, h, w)) < 0.4] = np.inf
    depth[:, :5, :] = np.inf                                   # rows no layer covers
    a = rng.uniform(0.0, 0.6, size=(n_layers, h, w, 1)).astype(np.float32)
    rgba = np.concatenate([rng.uniform(0.0, 1.0, size=(n_layers, h, w, 3)).astype(np.float32) * a, a], axis=-1)
    rgba[np.isinf(depth)] = 5.0                                # garbage where a layer does not cover the pixel
    d_rgba = [torch.from_numpy(np.ascontiguousarray(rgba[l])).cuda() for l in range(n_layers)]
    d_dep = [torch.from_numpy(np.ascontiguousarray(depth[l])).cuda() for l in range(n_layers)]
    out = torch.full((h, w, 4), np.nan, device="cuda")
    ctx.composite([t.data_ptr() for t in d_rgba], [t.data_ptr() for t in d_dep], w, h, out.data_ptr())
    got = out.cpu().numpy().astype(np.float64)
    ref = np.zeros((h, w, 4))
    for j in range(h):
        for i in range(w):
            order = sorted((float(depth[l, j, i]), l) for l in range(n_layers) if np.isfinite(depth[l, j, i]))
            C = np.zeros(4)
            for _, l in order:
                C = C + (1.0 - C[3]) * rgba[l, j, i].astype(np.float64)
            ref[j, i] = C
    assert np.all(got[:5] == 0.0)
    assert np.abs(got - ref).max() < 1e-6, np.abs(got - ref).max()
