"""GPU parity: the HIP ray caster against the FP64 oracle, through the C ABI.

Every image is compared channel by channel with the oracle (2e-3 plus the
oracle's allowance for decisions within the margin); sample counts are
compared exactly in runs without early termination.
"""

import dataclasses

import numpy as np
import pytest

import oracle
import pins
from oracle.oracle import NO_TERMINATION
from parity import compare, log, pixel_list
from scenes import configs, fields, make_source, relayout
from scenes.layout import Scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1611_09048_amd import Context
    assert torch.cuda.is_available()
    c = Context(device=0)
    yield c
    c.close()


def gpu_render(ctx, scene, **kw):
    from paper_1611_09048_amd import device
    log("gpu render:", scene.label or scene.dims, scene.width, "x", scene.height, kw)
    img, cnt = device.render_scene(ctx, scene, **kw)
    return img, cnt


def full_parity(ctx, scene, label, counts=True, max_flagged=0.02):
    """Every pixel against the oracle, with and without early termination.  At most
    max_flagged of the pixels may carry a decision within its margin (the rest are held
    to the plain tolerance)."""
    img, cnt = gpu_render(ctx, scene)
    rec = oracle.render(scene)
    st = compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=label)
    assert st["flagged_pixels"] <= max_flagged * st["pixels"], (label, st["flagged_pixels"], st["pixels"])
    if counts:
        img2, cnt2 = gpu_render(ctx, scene, ert_threshold=NO_TERMINATION)
        rec2 = oracle.render(scene, ert_threshold=NO_TERMINATION)
        st2 = compare(img2.reshape(-1, 4), cnt2.reshape(-1), rec2, label=label + " no-termination")
        assert st2["flagged_pixels"] <= max_flagged * st2["pixels"], (label, st2["flagged_pixels"])
    return img, cnt, rec


def test_plain_scalar_full_size(ctx):
    """One scalar, 64^3, nearest, 256x256 (the full plain-caster workload)."""
    sc = configs.plain_scalar()
    _, _, rec = full_parity(ctx, sc, "plain_scalar")
    assert rec["samples"].sum() > 5e5


@pytest.mark.parametrize("direction", [configs.D0, (-1.0, 0.0, 0.0), (0.3, -0.9, -0.4), (0.0, 0.0, 1.0)])
def test_pic3_small(ctx, direction):
    """Three sources, trilinear, two clip planes; 48^3, 300x170 (ragged against every tile shape)."""
    sc = configs.pic3(n=48, width=300, height=170, direction=direction)
    full_parity(ctx, sc, f"pic3 48^3 dir={direction}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_pic3_reduced_precision_storage(ctx, dtype):
    """FP16/BF16 storage: parity against the oracle on the stored values; error vs FP32 reported."""
    sc = configs.pic3(n=48, width=300, height=170, dtype=dtype)
    img, cnt, rec = full_parity(ctx, sc, f"pic3 48^3 {dtype}")
    ref32 = oracle.render(configs.pic3(n=48, width=300, height=170, dtype="f32"))
    d = np.abs(img.reshape(-1, 4).astype(np.float64) - ref32["rgba"])
    log(f"{dtype} storage vs FP32-field oracle: max {d.max(axis=0).tolist()} rms {np.sqrt((d ** 2).mean(axis=0)).tolist()}")


@pytest.mark.parametrize("chunk", range(4))
def test_random_small_scenes(ctx, chunk):
    """Random tiny scenes covering every feature (layouts, dtypes, chains, clips, cameras, thresholds)."""
    for seed in range(chunk * 15, chunk * 15 + 15):
        sc = configs.random_small_scene(seed)
        img, cnt = gpu_render(ctx, sc)
        rec = oracle.render(sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=f"random_small[{seed}]")
        img2, cnt2 = gpu_render(ctx, sc, ert_threshold=NO_TERMINATION)
        rec2 = oracle.render(sc, ert_threshold=NO_TERMINATION)
        compare(img2.reshape(-1, 4), cnt2.reshape(-1), rec2, label=f"random_small[{seed}] no-termination")


def bench_shape(ctx, sc):
    """Set the committed tuned tile shape the benchmark uses for this scene's size
    class and storage type; returns a function that restores the previous one."""
    import os
    from paper_1611_09048_amd import autotune
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = autotune.load_cache(os.path.join(root, "paper_1611_09048_amd", "tuned_gfx950.json"))
    cls = autotune.size_class(sc.width, sc.height)
    shape = cache.get(autotune.cache_key("gfx950", str(cls), f"pic3:{sc.sources[0].dtype}"))
    old = ctx.get_tile_shape(cls)
    if shape is not None:
        ctx.set_tile_shape(cls, *shape)
    log("tile shape", cls, shape)
    return lambda: ctx.set_tile_shape(cls, *old)


def test_pic3_full_size_sampled(ctx):
    """256^3, three sources, 1920x1080 in the benchmark's launch configuration (its
    tuned tile shape, derived volume); sampled pixels."""
    sc = configs.pic3()
    restore = bench_shape(ctx, sc)
    try:
        img, cnt = gpu_render(ctx, sc)
    finally:
        restore()
    rng = np.random.default_rng(0)
    px = pixel_list(sc.height, sc.width, 1500, rng, extra_rows=(540,), extra_cols=(960,),
                    hit_mask=img[..., 3] > 0, n_hit=2500)
    rec = oracle.render_pixels(sc, px)
    g = img[px[:, 1], px[:, 0]]
    c = cnt[px[:, 1], px[:, 0]]
    stats = compare(g, c, rec, label="pic3 256^3 1080p sampled")
    assert stats["samples"] > 1e5
    # image outside the sampled set: finite and in range
    assert np.isfinite(img).all() and img.min() >= 0.0 and img.max() <= 1.0 + 1e-6


def _host_threads():
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


@pytest.mark.parametrize("direction", [(-1.0, -1.0, -1.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0)])
def test_pic3_full_size_views(ctx, direction):
    """The benchmark frame as it is timed: 256^3, three sources, 1920x1080, one of the
    26 views (a diagonal, the +x axis, the +z axis), the benchmark's tuned tile shape and
    derived volume.  Every pixel and every sample count against the oracle (on host
    threads); at most 2 % of the pixels may carry a decision within its margin."""
    assert tuple(direction) in configs.views26()
    base = configs.pic3()
    sc = base.with_(camera=configs.orbit_camera(base.dims, direction))
    restore = bench_shape(ctx, sc)
    try:
        img, cnt = gpu_render(ctx, sc)
    finally:
        restore()
    rec = oracle.render(sc, threads=_host_threads())
    stats = compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=f"pic3 256^3 1080p view {direction}")
    assert stats["flagged_pixels"] <= 0.02 * stats["pixels"], stats
    assert stats["samples"] > 5e6


def test_pic3_4k_sampled(ctx):
    """The benchmark volume at 3840x2160 (four times the pixels and tiles of 1080p); sampled pixels."""
    sc = configs.pic3(width=3840, height=2160, direction=(0.3, 0.5, -0.8))
    restore = bench_shape(ctx, sc)
    try:
        img, cnt = gpu_render(ctx, sc)
    finally:
        restore()
    rng = np.random.default_rng(4)
    px = pixel_list(sc.height, sc.width, 1000, rng, extra_rows=(1080, 2159), extra_cols=(1920, 3839),
                    hit_mask=img[..., 3] > 0, n_hit=2000)
    rec = oracle.render_pixels(sc, px)
    stats = compare(img[px[:, 1], px[:, 0]], cnt[px[:, 1], px[:, 0]], rec, label="pic3 256^3 4K sampled")
    assert stats["samples"] > 1e5
    assert np.isfinite(img).all()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_pic3_reduced_precision_full_size_sampled(ctx, dtype):
    """The benchmark scene with FP16 / BF16 storage at 256^3, 1920x1080, in the
    benchmark's launch configuration: parity against the oracle on the stored
    values at sampled pixels, and the per-channel max and RMS error against the
    oracle of the FP32 fields reported beside the FP32-storage run's."""
    sc = configs.pic3(dtype=dtype)
    sc32 = configs.pic3()
    rng = np.random.default_rng(7)
    restore = bench_shape(ctx, sc)
    try:
        img, cnt = gpu_render(ctx, sc)
    finally:
        restore()
    restore = bench_shape(ctx, sc32)
    try:
        img32, _ = gpu_render(ctx, sc32)
    finally:
        restore()
    px = pixel_list(sc.height, sc.width, 600, rng, extra_rows=(540,), hit_mask=img[..., 3] > 0, n_hit=1500)
    rec = oracle.render_pixels(sc, px)
    g = img[px[:, 1], px[:, 0]]
    stats = compare(g, cnt[px[:, 1], px[:, 0]], rec, label=f"pic3 256^3 1080p {dtype} sampled")
    assert stats["samples"] > 5e4
    ref32 = oracle.render_pixels(sc32, px)["rgba"].reshape(-1, 4)
    for name, v in ((dtype, g), ("f32", img32[px[:, 1], px[:, 0]])):
        d = np.abs(v.reshape(-1, 4).astype(np.float64) - ref32)
        log(f"{name} storage vs FP32-field oracle (1080p sampled): max {d.max(axis=0).tolist()} "
            f"rms {np.sqrt((d ** 2).mean(axis=0)).tolist()}")
    assert np.isfinite(img).all() and img.min() >= 0.0 and img.max() <= 1.0 + 1e-6


def test_closed_form_slab_on_gpu(ctx):
    """The constant-42 source behind add(-41.5), constant TF (a=0.1): A = 1 - 0.9^16 exactly in closed form."""
    dims = (8, 6, 5)
    src = make_source("const42", fields.constant(dims, 0, 42.0), guard=0, chain="add(-41.5)",
                      tf=configs.constant_tf((0.2, 0.6, 0.9), 0.1))
    cam = configs.axis_camera(dims, axis=0, width=9, height=7, ortho_height=9.0)
    for interp in (0, 1):
        sc = Scene(dims=dims, sources=[src], camera=cam, width=9, height=7, step=0.5, interpolation=interp,
                   ert_threshold=NO_TERMINATION)
        img, cnt = gpu_render(ctx, sc)
        hit = cnt > 0
        assert np.array_equal(hit, pins._hit_mask(sc))
        assert np.all(cnt[hit] == 16)
        A = 1.0 - 0.9 ** 16
        assert np.allclose(img[hit][:, 3], A, atol=2e-6)
        assert np.allclose(img[hit][:, :3], np.array([0.2, 0.6, 0.9]) * A, atol=2e-6)
        assert np.all(img[~hit] == 0.0)


def test_transfer_table_ends_on_gpu(ctx):
    """Chain outputs at or beyond the ends of [0, 1] classify to the transfer function's end
    points exactly (a chain maps the data into the transfer function's domain, Sec. 3.3, and
    outputs outside [0, 1] are clamped to it): a constant
    source read through add(c) gives 16 identical scan points per ray, so A = 1 - (1 - a)^16
    and RGB = rgb * A in closed form, with (rgb, a) the first or the last control point."""
    dims = (8, 6, 5)
    first, last = (0.0, 0.1, 0.2, 0.3, 0.05), (1.0, 0.7, 0.55, 0.25, 0.08)
    tf = [first, (0.37, 0.9, 0.1, 0.5, 0.2), last]
    cam = configs.axis_camera(dims, axis=0, width=9, height=7, ortho_height=9.0)
    for chain, end in (("add(-41)", last), ("add(-40.3)", last), ("add(-42)", first), ("add(-45)", first)):
        src = make_source("const42", fields.constant(dims, 0, 42.0), guard=0, chain=chain, tf=tf)
        for interp in (0, 1):
            sc = Scene(dims=dims, sources=[src], camera=cam, width=9, height=7, step=0.5, interpolation=interp,
                       ert_threshold=NO_TERMINATION)
            img, cnt = gpu_render(ctx, sc)
            hit = cnt > 0
            assert np.array_equal(hit, pins._hit_mask(sc)) and np.all(cnt[hit] == 16), chain
            a = float(np.float32(end[4]))
            A = 1.0 - (1.0 - a) ** 16
            assert np.allclose(img[hit][:, 3], A, atol=2e-6), (chain, interp)
            rgb = np.array(end[1:4], dtype=np.float32).astype(np.float64)
            assert np.allclose(img[hit][:, :3], rgb * A, atol=2e-6), (chain, interp)


# Chains of exactly 8 functors (the interface's maximum) for sources of 1 to 4 components.
_MAX_CHAINS = {
    1: "mul(1.5) | add(0.25) | pow(2) | mul(0.5) | add(-0.125) | mul(2) | add(0.1) | mul(0.75)",
    2: "mul(0.5, 1.5) | add(0.25) | pow(2) | add(-0.1, 0.2) | mul(1.25) | sum | mul(0.5) | add(0.05)",
    3: "mul(2, 3, 4) | add(1) | mul(0.1) | pow(2) | add(-0.2, 0.1, 0) | length | mul(0.6) | add(-0.05)",
    4: "add(0.5) | mul(0.25, 0.5, 0.75, 1) | pow(2) | add(0.1) | mul(1.5) | sum | mul(0.2) | pow(0.5)",
}


def _maximum_scene(interpolation):
    """8 sources (1 to 4 components, FP32/FP16/BF16, AoS and SoA, with and without guard
    layers), each behind an 8-functor chain, and 8 clipping planes: every per-render limit
    of the interface at once (Sec. 3.2 sources, Sec. 3.3 chains)."""
    rng = np.random.default_rng(811)
    dims = (14, 12, 10)
    srcs = []
    for s in range(8):
        f_dim = 1 + s % 4
        guard = s % 2
        vals = fields.uniform_random(rng, dims, guard, f_dim, -1.0, 1.5)
        srcs.append(make_source(f"s{s}", vals, dtype=("f32", "f16", "bf16")[s % 3], guard=guard,
                                chain=_MAX_CHAINS[f_dim], weight=float(rng.uniform(0.2, 1.0)),
                                tf=configs.random_tf(rng, 5, 0.3), layout=("aos", "soa")[(s // 2) % 2]))
    # 8 planes, each keeping the side of the centre within 0.3 of the box diagonal along a
    # random normal: every plane cuts, and a region around the centre stays
    c = np.array(dims, dtype=np.float64) / 2.0
    r = 0.3 * float(np.linalg.norm(dims))
    clip = []
    for _ in range(8):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        clip.append((float(-n[0]), float(-n[1]), float(-n[2]), float(n @ c + r)))
    cam = configs.orbit_camera(dims, (0.3, -0.8, 0.5))
    return Scene(dims=dims, sources=srcs, camera=cam, width=96, height=72, step=0.5,
                 interpolation=interpolation, clip=clip, ert_threshold=0.999, label=f"maximums interp={interpolation}")


@pytest.mark.parametrize("interpolation", [0, 1])
def test_interface_maximums(ctx, interpolation):
    """Every pixel and sample count against the oracle at the interface's per-render maximums."""
    sc = _maximum_scene(interpolation)
    img, cnt, rec = full_parity(ctx, sc, sc.label, max_flagged=0.05)
    assert (cnt > 0).sum() > 200, "the clipped volume should still cover some pixels"


def _pic3_variant(sc, **src_changes):
    srcs = [dataclasses.replace(s, **src_changes) for s in sc.sources]
    return sc.with_(sources=srcs)


def test_layout_invariance_bitwise(ctx):
    """AoS, SoA, padded pitch, permuted and reversed axes give the same image bit for bit."""
    sc = configs.pic3(n=32, width=160, height=96)
    ref, refc = gpu_render(ctx, sc)
    layouts = [dict(layout="soa"), dict(order=(2, 0, 1)), dict(flip=(True, False, True)),
               dict(layout="soa", order=(1, 2, 0), flip=(False, True, False), pitch_align=4),
               dict(pitch_align=1024)]
    for lk in layouts:
        s2 = sc.with_(sources=[relayout(s, **lk) for s in sc.sources])
        img, cnt = gpu_render(ctx, s2)
        assert np.array_equal(img, ref), lk
        assert np.array_equal(cnt, refc), lk


def test_disabled_and_zero_weight_sources(ctx):
    """A disabled source (even with NULL data) and a zero-weight source equal the source being absent."""
    sc = configs.pic3(n=32, width=120, height=80)
    absent = sc.with_(sources=sc.sources[:2])
    ref, _ = gpu_render(ctx, absent)
    disabled = sc.with_(sources=sc.sources[:2] + [dataclasses.replace(sc.sources[2], enabled=False)])
    img, _ = gpu_render(ctx, disabled)
    assert np.array_equal(img, ref)
    zero = sc.with_(sources=sc.sources[:2] + [dataclasses.replace(sc.sources[2], weight=0.0)])
    img, _ = gpu_render(ctx, zero)
    assert np.array_equal(img, ref)
    # disabled with NULL component pointers
    from paper_1611_09048_amd import device
    import torch
    vol = device.upload_volume(ctx, absent, 0)
    descs = list(vol.descs)
    from paper_1611_09048_amd import binding
    descs.append(binding.source_desc(name="null", f_dim=3, dtype="f32", comp=[0, 0, 0], stride=(12, 0, 0), guard=1,
                                     enabled=False))
    ctx.set_sources(0, absent.dims, descs)
    for k, s in enumerate(absent.sources):
        ctx.set_transfer(0, k, s.tf)
    out = device.new_image(absent)
    ctx.render([device.render_job(absent, 0, out)])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)


def test_guard_poison_never_reaches_image(ctx):
    """NaN just outside the declared guard (and in an undeclared guard) never reaches a pixel."""
    rng = np.random.default_rng(21)
    dims = (20, 17, 23)
    vals = fields.uniform_random(rng, dims, 1, 3, -0.5, 0.5)
    tf = configs.random_tf(rng, 6, 0.2)
    base = make_source("v", vals, guard=1, chain="length", tf=tf)
    poisoned = make_source("v", vals, guard=1, chain="length", tf=tf, extra_layers=2)
    cam = configs.orbit_camera(dims, (0.7, -0.2, 0.5), 1.2, 70.0)
    sc = Scene(dims=dims, sources=[base], camera=cam, width=64, height=48, interpolation=1)
    a, _ = gpu_render(ctx, sc)
    b, _ = gpu_render(ctx, sc.with_(sources=[poisoned]))
    assert np.isfinite(b).all() and np.array_equal(a, b)
    # declared guard 0 over a NaN layer: clamps to the border instead of reading it
    g0 = make_source("v", vals[1:-1, 1:-1, 1:-1], guard=0, chain="length", tf=tf, extra_layers=1)
    inner = make_source("v", vals[1:-1, 1:-1, 1:-1], guard=0, chain="length", tf=tf)
    c, _ = gpu_render(ctx, sc.with_(sources=[g0]))
    d, _ = gpu_render(ctx, sc.with_(sources=[inner]))
    assert np.isfinite(c).all() and np.array_equal(c, d)


def test_fp16_exact_values_bitwise(ctx):
    """Values exactly representable in FP16 render bit-identically from FP16 and FP32 storage."""
    rng = np.random.default_rng(8)
    dims = (24, 20, 18)
    v = (rng.integers(0, 256, size=(dims[2] + 2, dims[1] + 2, dims[0] + 2, 3)) / 256.0).astype(np.float32)
    tf = configs.random_tf(rng, 6, 0.1)
    cam = configs.orbit_camera(dims, (0.4, 1.0, -0.3))
    for dt in ("f16", "bf16"):
        a = make_source("v", v, guard=1, chain="length | mul(0.7)", tf=tf)
        b = make_source("v", v, dtype=dt, guard=1, chain="length | mul(0.7)", tf=tf)
        sc = Scene(dims=dims, sources=[a], camera=cam, width=80, height=64, interpolation=1)
        ia, _ = gpu_render(ctx, sc)
        ib, _ = gpu_render(ctx, sc.with_(sources=[b]))
        assert np.array_equal(ia, ib), dt


def test_early_termination_bound(ctx):
    """Stopping at theta moves a channel by at most 1 - theta (plus FP32 rounding)."""
    sc = configs.pic3(n=40, width=128, height=96)
    srcs = [dataclasses.replace(s, tf=[(x, r, g, b, min(1.0, 8 * a)) for (x, r, g, b, a) in s.tf])
            for s in sc.sources]
    sc = sc.with_(sources=srcs)
    full, _ = gpu_render(ctx, sc, ert_threshold=NO_TERMINATION)
    for theta in (0.999, 0.99, 0.9):
        cut, _ = gpu_render(ctx, sc, ert_threshold=theta)
        assert np.all(np.abs(cut.astype(np.float64) - full) <= (1.0 - theta) + 1e-5), theta


def test_tile_shapes_and_schedules(ctx):
    """Tile shape and unroll never change a pixel; lanes-per-ray schedules agree with the oracle."""
    sc = configs.pic3(n=32, width=203, height=77)
    ref, refc = gpu_render(ctx, sc)
    cls = 8                                  # size class of a 203-wide image: ceil(log2(203))
    rec = oracle.render(sc)
    try:
        for ww, wx, u in ((16, 2, 1), (32, 1, 1), (64, 4, 1), (8, 4, 2), (16, 1, 2)):
            ctx.set_tile_shape(cls, ww, wx, u, 1, 0)
            img, cnt = gpu_render(ctx, sc)
            assert np.array_equal(img, ref) and np.array_equal(cnt, refc), (ww, wx, u)
        for ww, wx, g, m in ((8, 2, 2, 0), (16, 1, 2, 0), (8, 4, 4, 0), (16, 2, 4, 4), (32, 1, 2, 0), (8, 1, 8, 0),
                             (4, 2, 16, 4), (8, 2, 8, 4), (4, 4, 16, 0), (8, 4, 1, 4), (2, 2, 32, 0), (1, 4, 32, 0),
                             (1, 1, 64, 0), (1, 4, 64, 0)):
            ctx.set_tile_shape(cls, ww, wx, 1, g, m)
            img, cnt = gpu_render(ctx, sc)
            compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=f"lanes={g} wave_w={ww} waves_x={wx} min_waves={m}")
            assert np.abs(img - ref).max() < 1e-5
            again, _ = gpu_render(ctx, sc)
            assert np.array_equal(again, img)
    finally:
        ctx.set_tile_shape(cls, 8, 2, 1, 1, 0)


def test_lanes_per_ray_full_parity(ctx):
    """Every feature under 2 to 64 lanes per ray (random tiny scenes) against the oracle."""
    try:
        for g in (2, 4, 16, 32, 64):
            for c in range(16):
                ctx.set_tile_shape(c, min(8, 64 // g), 2, 1, g, 0)
            for seed in range(20):
                sc = configs.random_small_scene(seed)
                img, cnt = gpu_render(ctx, sc)
                compare(img.reshape(-1, 4), cnt.reshape(-1), oracle.render(sc), label=f"random_small[{seed}] lanes={g}")
                img2, cnt2 = gpu_render(ctx, sc, ert_threshold=NO_TERMINATION)
                compare(img2.reshape(-1, 4), cnt2.reshape(-1), oracle.render(sc, ert_threshold=NO_TERMINATION),
                        label=f"random_small[{seed}] lanes={g} no-termination")
            sc = configs.pic3(n=48, width=300, height=170)
            full_parity(ctx, sc, f"pic3 48^3 lanes={g}")
    finally:
        for c in range(16):
            ctx.set_tile_shape(c, 8, 2, 1, 1, 0)


def test_tiny_and_ragged_images(ctx):
    base = configs.pic3(n=16, width=1, height=1)
    for w, h in ((1, 1), (1, 37), (53, 1), (17, 3), (65, 65)):
        sc = base.with_(width=w, height=h)
        img, cnt = gpu_render(ctx, sc)
        rec = oracle.render(sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=f"ragged {w}x{h}")


def _degenerate_scenes():
    """(label, scene, expect_empty) for the method's degenerate inputs."""
    rng = np.random.default_rng(97)
    out = []
    for dims in ((1, 9, 7), (13, 1, 1), (6, 5, 1), (1, 1, 1)):
        for guard in (0, 1):
            vals = fields.uniform_random(rng, dims, guard, 3, -1.0, 1.5)
            src = make_source("v", vals, guard=guard, chain="length | mul(0.7)", weight=1.0,
                              tf=configs.random_tf(rng, 4, 0.6))
            for interp in (0, 1):
                cam = configs.orbit_camera(dims, (0.4, -0.7, 0.6), distance_factor=2.5)
                out.append((f"thin {dims} guard={guard} interp={interp}",
                            Scene(dims=dims, sources=[src], camera=cam, width=21, height=17, step=0.5,
                                  interpolation=interp), False))
    base = configs.pic3(n=16, width=40, height=30)
    c = np.array(base.dims, dtype=np.float64) / 2.0
    # two opposite planes whose kept sides do not meet: nothing is kept
    out.append(("clipped away", base.with_(clip=[(1.0, 0.0, 0.0, -(c[0] + 3.0)), (-1.0, 0.0, 0.0, c[0] - 3.0)]),
                True))
    # a camera whose view points away from the box
    away = configs.orbit_camera(base.dims, (0.3, 0.5, -0.8))
    back = dataclasses.replace(away, center=tuple(2.0 * np.array(away.eye) - np.array(away.center)))
    out.append(("looking away", base.with_(camera=back), True))
    out.append(("termination threshold 1e-6", base.with_(ert_threshold=1e-6), False))
    out.append(("step longer than the box", base.with_(step=40.0), False))
    return out


def test_degenerate_inputs(ctx):
    """Volumes one cell thick (and a single cell), with and without guard layers; clip planes
    that keep nothing; a camera looking away from the box; a termination threshold of 1e-6
    (a ray ends at its first scan point of any opacity); a step longer than the box (at most one
    scan point): every pixel and sample count against the oracle, and the empty cases empty.
    A threshold of 0 is the interface's default, 0.999: the same image bit for bit."""
    base = configs.pic3(n=16, width=40, height=30)
    d0, c0 = gpu_render(ctx, base.with_(ert_threshold=0.0))
    d1, c1 = gpu_render(ctx, base.with_(ert_threshold=0.999))
    assert np.array_equal(d0, d1) and np.array_equal(c0, c1)
    for label, sc, empty in _degenerate_scenes():
        img, cnt = gpu_render(ctx, sc)
        rec = oracle.render(sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=label)
        if empty:
            assert np.all(cnt == 0) and np.all(img == 0.0), label
        else:
            assert (cnt > 0).any(), label


def test_mirror_symmetry(ctx):
    """A field mirror-symmetric in y seen from the mirror plane gives a left-right mirrored image."""
    rng = np.random.default_rng(5)
    dims = (31, 24, 26)
    # rows y = -1..11 (guard included), mirrored onto y = 12..24 about the plane y = 12
    half = rng.uniform(0.0, 1.0, size=(dims[2] + 2, 13, dims[0] + 2)).astype(np.float32)
    v = np.concatenate([half, half[:, ::-1, :]], axis=1)
    src = make_source("m", v, guard=1, tf=configs.random_tf(rng, 5, 0.2))
    from scenes import Camera
    cam = Camera(eye=(-40.0, 12.0, 30.0), center=(15.5, 12.0, 13.0), up=(0.0, 0.0, 1.0), fovy_deg=45.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=100, height=70, interpolation=1)
    img, _ = gpu_render(ctx, sc)
    assert img[..., 3].max() > 0.05
    assert np.allclose(img, img[:, ::-1], atol=2e-3)


def test_screen_rectangle_culling_is_conservative(ctx):
    """Rays outside the box's projected rectangle are skipped: for cameras that put
    the box at the image border, partly off screen, very close (corners behind
    the eye) or far, every pixel with samples in the oracle has them on the GPU."""
    rng = np.random.default_rng(77)
    base = configs.plain_scalar(n=12, width=40, height=30)
    dims = np.array(base.dims, dtype=np.float64)
    for k in range(24):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        dist = float(rng.choice([0.3, 0.9, 1.5, 4.0, 12.0])) * np.linalg.norm(dims)
        centre = dims / 2 + rng.uniform(-0.6, 0.6, size=3) * dims     # aim off-centre: box near the border
        eye = centre + dist * d
        ortho = k % 4 == 3
        up = (0.0, 0.0, 1.0) if abs(d[2]) < 0.9 else (0.0, 1.0, 0.0)
        from scenes import Camera
        cam = Camera(eye=tuple(eye), center=tuple(centre), up=up, fovy_deg=float(rng.uniform(20, 100)),
                     projection="orthographic" if ortho else "perspective", ortho_height=float(rng.uniform(6, 30)))
        sc = base.with_(camera=cam, width=int(rng.integers(7, 48)), height=int(rng.integers(5, 40)))
        img, cnt = gpu_render(ctx, sc)
        rec = oracle.render(sc)
        compare(img.reshape(-1, 4), cnt.reshape(-1), rec, label=f"culling camera {k}")
