"""Checks that pin the CPU oracle to facts fixed outside it.

Each check takes an oracle library handle (the normal build or a deliberately
broken copy) and raises AssertionError when the oracle disagrees with:
  - closed forms: a constant slab composites to 1-(1-a)^n, an affine field
    seen along an axis gives a finite product known without any grid access;
  - the paper's worked functor chains (Sec. 3.3) and the dimension changes
    of Tab. 'functors';
  - ray/box geometry special cases and the pixel count of an axis projection;
  - an independent brute-force per-sample loop on tiny grids;
  - the bound that early termination at theta moves a channel by at most 1-theta.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle
from oracle import brute
from scenes import Camera, Scene, make_source
from scenes import configs, fields

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _img(rec, sc):
    return rec["rgba"].reshape(sc.height, sc.width, 4)


def _cnt(rec, sc):
    return rec["samples"].reshape(sc.height, sc.width)


# ---------------------------------------------------------------------------
# P1: constant slab
# ---------------------------------------------------------------------------

def _slab_scene(L=8, a=0.1, rgb=(0.2, 0.6, 0.9), weight=1.0, interpolation=0, guard=0, step=0.5,
                ert=1.0, clip=(), extra_sources=()):
    dims = (L, 6, 5)
    # the paper's analytic example source is 42 everywhere; add(-41.5) brings it into [0,1]
    src = make_source("const42", fields.constant(dims, guard, 42.0), guard=guard, chain="add(-41.5)",
                      weight=weight, tf=configs.constant_tf(rgb, a))
    cam = configs.axis_camera(dims, axis=0, width=9, height=7, ortho_height=9.0)
    return Scene(dims=dims, sources=[src, *extra_sources], camera=cam, width=9, height=7, step=step,
                 interpolation=interpolation, clip=list(clip), ert_threshold=ert)


def _hit_mask(sc):
    """Pixels of the axis camera whose ray runs through the box (pixel centres strictly inside)."""
    cam = sc.camera
    h = cam.ortho_height / 2.0
    mask = np.zeros((sc.height, sc.width), dtype=bool)
    for j in range(sc.height):
        for i in range(sc.width):
            x = (2.0 * (i + 0.5) / sc.width - 1.0) * h * sc.width / sc.height
            y = (1.0 - 2.0 * (j + 0.5) / sc.height) * h
            # axis 0 camera: right = fwd x up = (1,0,0)x(0,0,1) = (0,-1,0), up' = (0,0,1)
            py = cam.center[1] - x
            pz = cam.center[2] + y
            mask[j, i] = 0.0 < py < sc.dims[1] and 0.0 < pz < sc.dims[2]
    return mask


def pin_constant_slab(lib):
    for interp, guard in ((0, 0), (1, 0), (1, 1)):
        sc = _slab_scene(interpolation=interp, guard=guard)
        rec = oracle.render(sc, lib=lib)
        img, cnt = _img(rec, sc), _cnt(rec, sc)
        hit = _hit_mask(sc)
        assert hit.sum() > 10 and (~hit).sum() > 4
        n = 16                                    # L / step
        A = 1.0 - (1.0 - 0.1) ** n
        assert np.all(cnt[hit] == n), (interp, guard, cnt)
        assert np.all(cnt[~hit] == 0)
        assert np.allclose(img[hit][:, 3], A, rtol=0, atol=1e-12)
        assert np.allclose(img[hit][:, :3], np.array([0.2, 0.6, 0.9]) * A, rtol=0, atol=1e-12)
        assert np.all(img[~hit] == 0.0)


def pin_constant_slab_weight_and_two_sources(lib):
    dims = (8, 6, 5)
    second = make_source("const42b", fields.constant(dims, 0, 42.0), guard=0, chain="add(-41.5)",
                         weight=0.5, tf=configs.constant_tf((1.0, 0.0, 0.25), 0.3))
    sc = _slab_scene(weight=0.8, extra_sources=[second])
    rec = oracle.render(sc, lib=lib)
    img = _img(rec, sc)
    hit = _hit_mask(sc)
    S = 0.8 * 0.1 + 0.5 * 0.3
    E = 0.8 * 0.1 * np.array([0.2, 0.6, 0.9]) + 0.5 * 0.3 * np.array([1.0, 0.0, 0.25])
    A = 1.0 - (1.0 - S) ** 16
    assert np.allclose(img[hit][:, 3], A, atol=1e-12)
    assert np.allclose(img[hit][:, :3], E / S * A, atol=1e-12)
    # a disabled source contributes nothing (and is never read: give it a NULL-free poisoned layout)
    second.enabled = False
    rec2 = oracle.render(sc, lib=lib)
    ref = oracle.render(_slab_scene(weight=0.8), lib=lib)
    assert np.array_equal(rec2["rgba"], ref["rgba"])
    # weight 0 is the same as the source being absent
    second.enabled = True
    second.weight = 0.0
    rec3 = oracle.render(sc, lib=lib)
    assert np.allclose(rec3["rgba"], ref["rgba"], atol=1e-15)


def pin_mix_saturation(lib):
    """Sources whose weighted opacities sum past 1 are rescaled to opacity 1."""
    dims = (8, 6, 5)
    second = make_source("b", fields.constant(dims, 0, 42.0), guard=0, chain="add(-41.5)", weight=1.0,
                         tf=configs.constant_tf((1.0, 0.0, 0.0), 0.9))
    sc = _slab_scene(a=0.6, rgb=(0.0, 0.0, 1.0), extra_sources=[second])
    rec = oracle.render(sc, lib=lib)
    img, cnt = _img(rec, sc), _cnt(rec, sc)
    hit = _hit_mask(sc)
    S = 0.6 + 0.9
    E = (0.6 * np.array([0.0, 0.0, 1.0]) + 0.9 * np.array([1.0, 0.0, 0.0])) / S
    assert np.allclose(img[hit][:, 3], 1.0, atol=1e-12)
    assert np.allclose(img[hit][:, :3], E, atol=1e-12)
    assert np.all(cnt[hit] == 1)                   # opacity 1 after the first sample meets theta = 1


def pin_constant_slab_ert(lib):
    sc = _slab_scene(L=40, ert=0.999)
    rec = oracle.render(sc, lib=lib)
    img, cnt = _img(rec, sc), _cnt(rec, sc)
    hit = _hit_mask(sc)
    n_star = math.ceil(math.log(0.001) / math.log(0.9))
    assert n_star == 66
    assert np.all(cnt[hit] == n_star), np.unique(cnt[hit])
    assert np.allclose(img[hit][:, 3], 1.0 - 0.9 ** n_star, atol=1e-12)


def pin_constant_slab_clip(lib):
    # keep x >= 3.1: samples at x = (k+1/2)/2 >= 3.1 are k = 6..15
    sc = _slab_scene(clip=[(1.0, 0.0, 0.0, -3.1)])
    rec = oracle.render(sc, lib=lib)
    cnt = _cnt(rec, sc)
    hit = _hit_mask(sc)
    n_kept = sum(1 for k in range(16) if (k + 0.5) * 0.5 >= 3.1)
    assert n_kept == 10
    assert np.all(cnt[hit] == n_kept)
    assert np.allclose(_img(rec, sc)[hit][:, 3], 1.0 - 0.9 ** n_kept, atol=1e-12)
    # a scaled normal describes the same half-space; the opposite plane keeps the rest
    sc2 = _slab_scene(clip=[(2.0, 0.0, 0.0, -6.2)])
    assert np.array_equal(oracle.render(sc2, lib=lib)["samples"], rec["samples"])
    sc3 = _slab_scene(clip=[(-1.0, 0.0, 0.0, 3.1)])
    assert np.all(_cnt(oracle.render(sc3, lib=lib), sc3)[hit] == 16 - n_kept)


# ---------------------------------------------------------------------------
# P2: linear ramp
# ---------------------------------------------------------------------------

def _ramp_scene(axis, sign, guard, L=12, alpha=0.0625, beta=0.03125, a_max=0.375, step=0.5):
    dims = [5, 6, 7]
    dims[axis] = L
    dims = tuple(dims)
    src = make_source("ramp", fields.ramp(dims, guard, alpha, beta, axis), guard=guard,
                      tf=configs.linear_alpha_tf((0.3, 0.5, 0.7), a_max))
    cam = configs.axis_camera(dims, axis=axis, sign=sign, width=6, height=6, ortho_height=4.0)
    return Scene(dims=dims, sources=[src], camera=cam, width=6, height=6, step=step, interpolation=1,
                 ert_threshold=1.0)


def pin_linear_ramp(lib):
    for axis in (0, 1, 2):
        for sign in (1.0, -1.0):
            for guard in (1, 0):
                L, alpha, beta, a_max = 12, 0.0625, 0.03125, 0.375   # exact in float32 storage
                sc = _ramp_scene(axis, sign, guard, L, alpha, beta, a_max)
                rec = oracle.render(sc, lib=lib)
                img, cnt = _img(rec, sc), _cnt(rec, sc)
                n = int(L / 0.5)
                # positions along the axis: the ray enters at 0 (sign +) or at L (sign -)
                ps = [(k + 0.5) * 0.5 if sign > 0 else L - (k + 0.5) * 0.5 for k in range(n)]
                if guard == 0:                     # clamp-to-edge within half a cell of each face
                    ps = [min(max(p, 0.5), L - 0.5) for p in ps]
                T, A = 1.0, 0.0
                for p in ps:
                    s = a_max * min(max(alpha * p + beta, 0.0), 1.0)
                    A = A + T * s
                    T = T * (1.0 - s)
                A_closed = 1.0 - np.prod([1.0 - a_max * min(max(alpha * p + beta, 0.0), 1.0) for p in ps])
                assert abs(A - A_closed) < 1e-14
                assert np.all(cnt == n), (axis, sign, guard, np.unique(cnt))
                assert np.allclose(img[..., 3], A_closed, rtol=0, atol=1e-12), (axis, sign, guard)
                assert np.allclose(img[..., :3], np.array([0.3, 0.5, 0.7]) * A_closed, atol=1e-12)


# ---------------------------------------------------------------------------
# P3: functor chains
# ---------------------------------------------------------------------------

def pin_functor_examples(lib):
    with open(os.path.join(GOLDEN, "functor_examples.json")) as f:
        g = json.load(f)
    for ex in g["examples"]:
        for case in ex["cases"]:
            v, _ = oracle.chain_eval(ex["chain"], ex["f_dim"], case["in"], lib=lib)
            assert abs(v - case["out"]) < 1e-12, (ex["id"], case, v)
    rng = np.random.default_rng(7)
    for _ in range(50):
        x, y, z = rng.uniform(-3, 3, size=3)
        v, d = oracle.chain_eval("mul(2,3,4) | add(1) | length", 3, [x, y, z], lib=lib)
        assert d == 1
        assert abs(v - math.sqrt((2 * x + 1) ** 2 + (3 * y + 1) ** 2 + (4 * z + 1) ** 2)) < 1e-12
        v, _ = oracle.chain_eval("mul(0,1,0) | sum", 3, [x, y, z], lib=lib)
        assert abs(v - y) < 1e-15
        v, _ = oracle.chain_eval("pow(2) | sum | pow(0.5)", 3, [x, y, z], lib=lib)
        assert abs(v - math.sqrt(x * x + y * y + z * z)) < 1e-12
        w = rng.uniform(0.1, 4.0)
        v, _ = oracle.chain_eval("pow(3) | pow(0.5)", 1, [w], lib=lib)
        assert abs(v - w ** 1.5) < 1e-12
        v, _ = oracle.chain_eval("", 4, [x, y, z, 1.0], lib=lib)
        assert v == x
    for case in g["dimension_changes"]["cases"]:
        _, d = oracle.chain_eval(case["chain"], case["f_dim"], [0.5] * case["f_dim"], lib=lib)
        assert d == case["dim"], case
    for bad, f_dim in (("foo", 1), ("add(1,2)", 3), ("length(2)", 3), ("add()", 1), ("mul(1) |", 1),
                       ("add(1 2)", 1), ("sum | add(1,2)", 2), (" | ".join(["add(1)"] * 9), 1),
                       ("add(1,2,3,4,5)", 4), ("length", 5)):
        try:
            oracle.chain_eval(bad, f_dim, [0.0] * 4, lib=lib)
        except ValueError:
            continue
        raise AssertionError(f"chain {bad!r} accepted")


def pin_chain_render_equivalence(lib):
    """mul(2) | pow(0.5) on f renders like the identity chain on sqrt(2 f) (nearest sampling)."""
    rng = np.random.default_rng(11)
    dims = (6, 7, 5)
    f = fields.uniform_random(rng, dims, 0, 1, 0.0, 0.4).astype(np.float64)
    tf = configs.random_tf(rng, 5, 0.5)
    cam = configs.orbit_camera(dims, (0.3, -1.0, 0.5), distance_factor=1.5, fovy_deg=50.0)
    a = make_source("f", f.astype(np.float32), guard=0, chain="mul(2) | pow(0.5)", tf=tf)
    b = make_source("g", np.sqrt(2.0 * a.values[..., 0]).astype(np.float32), guard=0, tf=tf)
    sa = Scene(dims=dims, sources=[a], camera=cam, width=11, height=9, interpolation=0)
    sb = sa.with_(sources=[b])
    ra, rb = oracle.render(sa, lib=lib), oracle.render(sb, lib=lib)
    assert np.array_equal(ra["samples"], rb["samples"])
    # sqrt(2f) stored as float32 differs from the chain's FP64 value by < 2^-24 relative
    assert np.allclose(ra["rgba"], rb["rgba"], atol=1e-6)
    assert ra["rgba"][:, 3].max() > 0.05


# ---------------------------------------------------------------------------
# P2b: transfer table
# ---------------------------------------------------------------------------

def pin_tf_table(lib):
    t = oracle.tf_table([(0.0, 0.1, 0.2, 0.3, 0.0), (1.0, 0.9, 0.7, 0.5, 1.0)], lib=lib)
    j = np.arange(256) / 255.0
    lin = np.stack([0.1 + 0.8 * j, 0.2 + 0.5 * j, 0.3 + 0.2 * j, j], axis=1)
    assert np.allclose(t, lin, atol=1e-15)
    pts = [(0.0, 0, 0, 0, 0), (51 / 255, 1.0, 0.5, 0.25, 0.125), (200 / 255, 0.0, 1.0, 0.0, 1.0), (1.0, 1, 1, 1, 1)]
    t = oracle.tf_table(pts, lib=lib)
    assert np.allclose(t[51], [1.0, 0.5, 0.25, 0.125], atol=1e-15)
    assert np.allclose(t[200], [0.0, 1.0, 0.0, 1.0], atol=1e-15)
    assert np.allclose(t[0], 0.0) and np.allclose(t[255], 1.0)
    w = 51.0 / 149.0                     # x = 102/255 lies 51/149 of the way from 51/255 to 200/255
    assert np.allclose(t[102], [1.0 - w, 0.5 + 0.5 * w, 0.25 - 0.25 * w, 0.125 + 0.875 * w], atol=1e-15)
    # halfway between two control points the table is their mean
    mid = oracle.tf_table([(0.0, 0, 0, 0, 0), (2 / 255, 1.0, 1.0, 1.0, 1.0), (1.0, 1, 1, 1, 1)], lib=lib)
    assert np.allclose(mid[1], 0.5, atol=1e-15)
    for bad in ([(0.0, 0, 0, 0, 0)], [(0.1, 0, 0, 0, 0), (1.0, 0, 0, 0, 0)], [(0.0, 0, 0, 0, 0), (0.9, 0, 0, 0, 0)],
                [(0.0, 0, 0, 0, 0), (0.5, 0, 0, 0, 0), (0.5, 0, 0, 0, 0), (1.0, 0, 0, 0, 0)],
                [(0.0, 0, 0, 0, 1.5), (1.0, 0, 0, 0, 0)]):
        try:
            oracle.tf_table(bad, lib=lib)
        except ValueError:
            continue
        raise AssertionError(f"transfer function {bad} accepted")


def pin_classification_lookup(lib):
    """A linear-alpha table classifies a constant value v to alpha = v (a slab of one sample)."""
    for v in (0.0, 0.2, 0.5, 0.73, 1.0, 1.7, -0.3):
        dims = (1, 3, 3)
        src = make_source("c", fields.constant(dims, 0, v), guard=0,
                          tf=configs.linear_alpha_tf((1.0, 1.0, 1.0), 1.0))
        cam = configs.axis_camera(dims, axis=0, width=3, height=3, ortho_height=3.0)
        sc = Scene(dims=dims, sources=[src], camera=cam, width=3, height=3, step=1.0, interpolation=0,
                   ert_threshold=1.0)
        rec = oracle.render(sc, lib=lib)
        centre = _img(rec, sc)[1, 1]
        assert _cnt(rec, sc)[1, 1] == 1
        assert abs(centre[3] - min(max(float(np.float32(v)), 0.0), 1.0)) < 1e-12, (v, centre)


# ---------------------------------------------------------------------------
# P5: geometry
# ---------------------------------------------------------------------------

def pin_geometry(lib):
    # axis projection: the number of hit pixels is the count of pixel centres over the box face
    dims = (5, 7, 3)
    src = make_source("c", fields.constant(dims, 0, 0.5), guard=0, tf=configs.constant_tf((1, 1, 1), 0.2))
    cam = configs.axis_camera(dims, axis=2, width=16, height=12, ortho_height=10.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=16, height=12, step=0.5, interpolation=0)
    rec = oracle.render(sc, lib=lib)
    cnt = _cnt(rec, sc)
    spacing = 10.0 / 12
    # axis 2 camera: fwd=(0,0,1), up=(0,1,0): right = fwd x up = (-1,0,0), up' = (0,1,0)
    cols = [i for i in range(16) if 0 < dims[0] / 2 - (i + 0.5 - 8) * spacing < dims[0]]
    rows = [j for j in range(12) if 0 < dims[1] / 2 + (6 - j - 0.5) * spacing < dims[1]]
    assert (cnt > 0).sum() == len(cols) * len(rows)
    assert np.all(cnt[np.ix_(rows, cols)] == int(dims[2] / 0.5))
    # eye inside the box: every ray hits, starts at t0 = 0 and leaves where the nearest face is
    cube = (8, 8, 8)
    src = make_source("c", fields.constant(cube, 0, 0.5), guard=0, tf=configs.constant_tf((1, 1, 1), 0.01))
    cam = Camera(eye=(4.0, 4.0, 4.0), center=(10.0, 5.0, 4.5), up=(0.0, 0.0, 1.0), fovy_deg=90.0)
    sc = Scene(dims=cube, sources=[src], camera=cam, width=7, height=5, step=0.5, interpolation=0,
               ert_threshold=1.0)
    rec = oracle.render(sc, lib=lib)
    for j in range(5):
        for i in range(7):
            hit, o, d, t0, t1 = oracle.ray(sc, i, j, lib=lib)
            assert hit and t0 == 0.0 and abs(np.linalg.norm(d) - 1.0) < 1e-14
            t_exit = min(4.0 / abs(c) for c in d if c != 0.0)
            assert abs(t1 - t_exit) < 1e-12
            n = sum(1 for k in range(100) if (k + 0.5) * 0.5 < t_exit)
            assert rec["samples"][j * 7 + i] == n
    # a ray parallel to a face and outside it misses; on the face plane it hits
    dims = (4, 4, 4)
    src = make_source("c", fields.constant(dims, 0, 0.5), guard=0, tf=configs.constant_tf((1, 1, 1), 0.2))
    for y, expect in ((4.5, False), (4.0, True), (-0.01, False), (2.0, True)):
        cam = Camera(eye=(-5.0, y, 2.0), center=(0.0, y, 2.0), up=(0.0, 0.0, 1.0), projection="orthographic",
                     ortho_height=1.0)
        sc = Scene(dims=dims, sources=[src], camera=cam, width=1, height=1, step=0.5, interpolation=0)
        hit, o, d, t0, t1 = oracle.ray(sc, 0, 0, lib=lib)
        assert hit == expect, (y, hit)
        assert (oracle.render(sc, lib=lib)["samples"][0] > 0) == expect
    # a perspective camera behind the box looking away sees nothing
    cam = Camera(eye=(-3.0, 2.0, 2.0), center=(-10.0, 2.0, 2.0), up=(0.0, 0.0, 1.0), fovy_deg=40.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=6, height=6, step=0.5, interpolation=0)
    assert np.all(oracle.render(sc, lib=lib)["rgba"] == 0.0)


def pin_orientation(lib):
    """Row 0 is the top of the image and the camera's right is fwd x up."""
    dims = (8, 8, 8)
    v = np.zeros((8, 8, 8), dtype=np.float32)
    v[6:, 0:2, :] = 1.0          # high z, low y: [z][y][x]
    src = make_source("o", v, guard=0, tf=configs.linear_alpha_tf((1, 1, 1), 0.5))
    # looking along +x with up +z: right = (1,0,0) x (0,0,1) = (0,-1,0), so low y is on the right
    cam = configs.axis_camera(dims, axis=0, width=8, height=8, ortho_height=8.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=8, height=8, step=0.5, interpolation=0)
    img = _img(oracle.render(sc, lib=lib), sc)
    lit = img[..., 3] > 0
    assert lit[:2, 6:].all() and not lit[2:, :].any() and not lit[:, :6].any(), lit.astype(int)


def pin_perspective_symmetry(lib):
    """A field mirror-symmetric in y, seen from a camera on the mirror plane, gives a mirrored image."""
    rng = np.random.default_rng(5)
    dims = (7, 6, 5)
    half = fields.uniform_random(rng, (7, 3, 5), 0, 1, 0.0, 1.0)
    v = np.concatenate([half, half[:, ::-1, :]], axis=1)
    src = make_source("m", v, guard=0, tf=configs.random_tf(rng, 4, 0.4))
    cam = Camera(eye=(-9.0, 3.0, 7.0), center=(3.5, 3.0, 2.5), up=(0.0, 0.0, 1.0), fovy_deg=45.0)
    for interp in (0, 1):
        sc = Scene(dims=dims, sources=[src], camera=cam, width=10, height=7, step=0.4, interpolation=interp)
        img = _img(oracle.render(sc, lib=lib), sc)
        assert img[..., 3].max() > 0.05
        assert np.allclose(img, img[:, ::-1], atol=1e-9), interp


# ---------------------------------------------------------------------------
# P4: brute force; P6: early-termination bound
# ---------------------------------------------------------------------------

def pin_brute_force(lib, seeds=range(40)):
    for seed in seeds:
        sc = configs.random_small_scene(seed)
        rec = oracle.render(sc, lib=lib)
        img, cnt = brute.render(sc)
        assert np.array_equal(_cnt(rec, sc), np.array(cnt)), seed
        assert np.allclose(_img(rec, sc), np.array(img), rtol=0, atol=1e-12, equal_nan=False), seed


def pin_ert_bound(lib):
    for seed in range(6):
        sc = configs.random_small_scene(100 + seed)
        for s in sc.sources:
            s.tf = [(x, r, g, b, min(1.0, 4 * a)) for (x, r, g, b, a) in s.tf]
        full = oracle.render(sc, lib=lib, ert_threshold=1.0)["rgba"]
        for theta in (0.999, 0.99, 0.9):
            cut = oracle.render(sc, lib=lib, ert_threshold=theta)["rgba"]
            assert np.all(np.abs(cut - full) <= (1.0 - theta) + 1e-12), (seed, theta)


def pin_fp16_bf16_reads(lib):
    """Values exactly representable in FP16 and BF16 render identically from either storage."""
    rng = np.random.default_rng(9)
    dims = (5, 4, 6)
    v = (rng.integers(0, 64, size=(6 + 2, 4 + 2, 5 + 2, 3)) / 64.0).astype(np.float32)
    tf = configs.random_tf(rng, 5, 0.6)
    base = make_source("v", v, guard=1, chain="length | mul(0.6)", tf=tf)
    cam = configs.orbit_camera(dims, (1.0, -0.4, 0.7), 1.4, 50.0)
    sc = Scene(dims=dims, sources=[base], camera=cam, width=9, height=8, interpolation=1)
    ref = oracle.render(sc, lib=lib)
    assert ref["rgba"][:, 3].max() > 0.05
    for dt in ("f16", "bf16"):
        s = make_source("v", v, dtype=dt, guard=1, chain="length | mul(0.6)", tf=tf)
        assert np.array_equal(s.values, base.values)
        r = oracle.render(sc.with_(sources=[s]), lib=lib)
        assert np.array_equal(r["rgba"], ref["rgba"]), dt
    # and a value that needs the exponent/mantissa split right: 1.5 * 2^-3 and 3 * 2^4
    for val in (0.1875, 48.0, 2.0 ** -20):
        for dt in ("f16", "bf16"):
            s = make_source("c", fields.constant((1, 1, 1), 0, val), dtype=dt, guard=0, chain="mul(0.01)",
                            tf=configs.linear_alpha_tf((1, 1, 1), 1.0))
            cam = configs.axis_camera((1, 1, 1), axis=0, width=1, height=1, ortho_height=0.5)
            sc1 = Scene(dims=(1, 1, 1), sources=[s], camera=cam, width=1, height=1, step=1.0,
                        interpolation=0, ert_threshold=1.0)
            a = oracle.render(sc1, lib=lib)["rgba"][0, 3]
            assert abs(a - min(val * 0.01, 1.0)) < 1e-12, (val, dt, a)


# ---------------------------------------------------------------------------
# iso-surface mode: affine ramp (exact crossing and normal), sphere (bound)
# ---------------------------------------------------------------------------

def _iso_ramp_scene(direction, iso, interpolation=1, width=7, height=5):
    dims = (16, 6, 6)
    src = make_source("ramp", fields.ramp(dims, 1, 0.0625, 0.03125, 0), guard=1,
                      tf=[(0.0, 0.2, 0.4, 0.6, 0.1), (1.0, 1.0, 0.8, 0.0, 0.9)])
    src.iso = iso
    c = np.array(dims, dtype=np.float64) / 2.0
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    eye = c - 20.0 * d
    up = (0.0, 0.0, 1.0)
    cam = Camera(eye=tuple(eye), center=tuple(c), up=up, projection="orthographic", ortho_height=2.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=width, height=height, step=0.5,
               interpolation=interpolation, ert_threshold=1.0, mode="iso")
    return sc


def pin_iso_plane(lib):
    iso = 0.5                                   # 0.0625 x + 0.03125 = 0.5  ->  x* = 7.5
    x_star = (iso - 0.03125) / 0.0625
    tf_rgb = np.array([0.2, 0.4, 0.6]) + iso * (np.array([1.0, 0.8, 0.0]) - np.array([0.2, 0.4, 0.6]))
    for direction, cos in (((1.0, 0.0, 0.0), 1.0), ((-1.0, 0.0, 0.0), 1.0), ((1.0, 0.0, 1.0), 2 ** -0.5)):
        sc = _iso_ramp_scene(direction, iso)
        rec = oracle.render(sc, lib=lib)
        img, cnt = _img(rec, sc), _cnt(rec, sc)
        centre = img[sc.height // 2, sc.width // 2]
        assert centre[3] == 1.0, (direction, centre)
        assert np.allclose(centre[:3], tf_rgb * (0.3 + 0.7 * cos), atol=1e-12), (direction, centre)
        if direction == (1.0, 0.0, 0.0):
            # samples at x = (k + 1/2)/2: the first at or past x* ends the ray
            k = next(k for k in range(64) if (k + 0.5) * 0.5 >= x_star)
            assert cnt[sc.height // 2, sc.width // 2] == k + 1
        assert np.all(img[..., 3] == 1.0)        # every ray crosses the plane
    # nothing crosses an iso value outside the field's range
    sc = _iso_ramp_scene((1.0, 0.0, 0.0), 5.0)
    assert np.all(oracle.render(sc, lib=lib)["rgba"] == 0.0)


def pin_iso_bilinear(lib):
    """v = a x + c x z + b is reproduced exactly by trilinear interpolation and by
    half-voxel central differences; along a ray parallel to x at height z0 it is
    linear, so the refined crossing x* = (iso - b) / (a + c z0) is exact, and the
    gradient (a + c z0, 0, c x*) fixes the shading through x*."""
    a_, c_, b_ = 0.0625, 0.015625, 0.125          # dyadic: every stored value is exact in FP32
    dims = (16, 6, 6)
    xs = np.arange(-1, 17) + 0.5
    zs = np.arange(-1, 7) + 0.5
    v = np.empty((8, 8, 18, 1))
    v[..., 0] = (a_ * xs[None, None, :] + c_ * xs[None, None, :] * zs[:, None, None] + b_) * np.ones((8, 8, 18))
    iso = b_ + (a_ + 3.0 * c_) * 5.1           # x* = 5.1 at z0 = 3, between the samples at 4.75 and 5.25
    src = make_source("bilinear", v, guard=1, tf=[(0.0, 0.9, 0.5, 0.1, 0.2), (1.0, 0.1, 0.5, 0.9, 0.7)])
    src.iso = iso
    tf_rgb = np.array([0.9, 0.5, 0.1]) + iso * (np.array([0.1, 0.5, 0.9]) - np.array([0.9, 0.5, 0.1]))
    for sign in (1.0, -1.0):
        eye = (8.0 - sign * 20.0, 3.0, 3.0)
        cam = Camera(eye=eye, center=(8.0, 3.0, 3.0), up=(0.0, 0.0, 1.0), projection="orthographic",
                     ortho_height=3.0)
        sc = Scene(dims=dims, sources=[src], camera=cam, width=3, height=5, step=0.5, interpolation=1,
                   ert_threshold=1.0, mode="iso")
        img = _img(oracle.render(sc, lib=lib), sc)
        for j in range(sc.height):
            for i in range(sc.width):
                hit, o, d, t0, t1 = oracle.ray(sc, i, j, lib=lib)
                assert hit and abs(d[0]) == 1.0
                z0 = o[2]
                x_star = (iso - b_) / (a_ + c_ * z0)
                g = np.array([a_ + c_ * z0, 0.0, c_ * x_star])
                cos = abs(g[0]) / np.linalg.norm(g)
                assert np.allclose(img[j, i, :3], tf_rgb * (0.3 + 0.7 * cos), rtol=0, atol=1e-12), (sign, i, j)
                assert img[j, i, 3] == 1.0
    # a clip plane keeping x >= 6 removes the crossing from every ray
    sc = sc.with_(clip=[(1.0, 0.0, 0.0, -6.0)])
    assert np.all(oracle.render(sc, lib=lib)["rgba"] == 0.0)


def pin_iso_sphere(lib):
    """|p - c|^2 through trilinear interpolation lies in [r^2, r^2 + 3/4]: the surface radius is bounded."""
    dims = (24, 24, 24)
    c = np.array([12.0, 12.0, 12.0])
    xs = np.arange(-1, 25) + 0.5
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    v = np.stack([X - c[0], Y - c[1], Z - c[2]], axis=-1)
    R = 8.0
    src = make_source("sphere", v.astype(np.float32), guard=1, chain="pow(2) | sum",
                      tf=configs.constant_tf((0.5, 0.5, 0.5), 1.0))
    src.iso = R * R
    cam = Camera(eye=(40.0, 12.0, 12.0), center=(12.0, 12.0, 12.0), up=(0.0, 0.0, 1.0), fovy_deg=30.0)
    sc = Scene(dims=dims, sources=[src], camera=cam, width=9, height=9, step=0.25, interpolation=1,
               ert_threshold=1.0, mode="iso")
    rec = oracle.render(sc, lib=lib)
    img = _img(rec, sc)
    assert img[4, 4, 3] == 1.0                  # the centre ray meets the sphere
    # along the centre ray (the x axis) the crossing lies between radius sqrt(R^2 - 3/4) and R
    # and the normal is radial, so the headlight term is close to 1
    assert img[4, 4, 0] > 0.5 * (0.3 + 0.7 * 0.99)
    hits = img[..., 3] == 1.0
    assert 10 <= hits.sum() <= 81
    assert not hits[0, 0] and not hits[0, 8]     # corner rays pass beside the sphere


# ---------------------------------------------------------------------------
# several correct results: the allowance of decisions taken within their margins
# ---------------------------------------------------------------------------
#
# Scan points on these axis-aligned orthographic rays sit at x = (k + 1/2) step
# exactly (the rays enter the box at x = 0 from x = -10).  Steps of the form
# m / 2^e with (k + 1/2) step = B +- 2^-13 put a scan point half a margin
# (delta = 2^-12) from a cell boundary, a clip plane or the box exit, or, with
# 2^-11, two margins away; every position is exact in binary.

_D = oracle.oracle.DELTA


def _two_cell_scene(dims_x, boundary, step):
    """Nearest sampling of a field that is 0.25 left of x = boundary and 0.75 right of it;
    linear alpha (a_max 0.5), rgb (0.2, 0.6, 0.9)."""
    dims = (dims_x, 3, 3)
    v = np.where(np.arange(dims_x) < boundary, 0.25, 0.75).astype(np.float32)
    v = np.broadcast_to(v[None, None, :], (3, 3, dims_x)).copy()
    src = make_source("step", v, guard=0, tf=configs.linear_alpha_tf((0.2, 0.6, 0.9), 0.5))
    cam = configs.axis_camera(dims, axis=0, width=3, height=3, ortho_height=3.0)
    return Scene(dims=dims, sources=[src], camera=cam, width=3, height=3, step=step, interpolation=0,
                 ert_threshold=1.0)


def pin_allowance_nearest_boundary(lib):
    # a cell with alpha 0.125 in front (T = 0.875), then a scan point 2^-13 from the boundary:
    # the other cell changes the colour by 0.9 * 0.25 and the opacity by 0.25
    expect = 0.875 * (0.9 * 0.25 + 0.25)
    for dims_x, boundary, step, label in ((2, 1, 2731 / 4096, "1 + 2^-13"), (3, 2, 5461 / 4096, "2 - 2^-13")):
        assert abs(1.5 * step - boundary) == 2.0 ** -13
        rec = oracle.render(_two_cell_scene(dims_x, boundary, step), lib=lib)
        assert np.all(rec["flags"] == 1) and np.all(rec["kinds"] == oracle.oracle.FLAG_NEAREST), label
        assert np.allclose(rec["allowance"], expect, rtol=0, atol=1e-12), (label, rec["allowance"])
        assert np.all(rec["count_slack"] == 0)
    # two margins from the boundary (1 + 2^-11): no decision is in doubt
    step = 683 / 1024
    assert 1.5 * step == 1.0 + 2 * _D
    rec = oracle.render(_two_cell_scene(2, 1, step), lib=lib)
    assert np.all(rec["flags"] == 0) and np.all(rec["allowance"] == 0.0), rec["allowance"]
    # trilinear sampling has no nearest-cell decision
    rec = oracle.render(_two_cell_scene(2, 1, 2731 / 4096).with_(interpolation=1), lib=lib)
    assert np.all(rec["flags"] == 0) and np.all(rec["allowance"] == 0.0)


def pin_allowance_clip_and_exit(lib):
    # trilinear: no nearest-cell decisions beside the ones under test
    a, rgb = 0.1, (0.2, 0.6, 0.9)
    contrib = max(rgb) * a + a                      # |E|max + S of one scan point of the slab
    eps = 2.0 ** -13
    # keep x <= 2.75 + eps: the scan point at 2.75 is kept half a margin inside, behind 5 others
    sc = _slab_scene(interpolation=1, clip=[(-1.0, 0.0, 0.0, 2.75 + eps)])
    rec, hit = oracle.render(sc, lib=lib), _hit_mask(sc).reshape(-1)
    assert np.all(_cnt(rec, sc).reshape(-1)[hit] == 6)
    assert np.allclose(rec["allowance"][hit], 0.9 ** 5 * contrib, rtol=0, atol=1e-12), rec["allowance"][hit]
    assert np.all(rec["count_slack"][hit] == 1) and np.all(rec["kinds"][hit] == oracle.oracle.FLAG_CLIP)
    assert np.all(rec["allowance"][~hit] == 0.0) and np.all(rec["flags"][~hit] == 0)
    # keep x >= 2.75 + eps: the same point is dropped half a margin outside, nothing in front
    sc = _slab_scene(interpolation=1, clip=[(1.0, 0.0, 0.0, -(2.75 + eps))])
    rec = oracle.render(sc, lib=lib)
    assert np.all(_cnt(rec, sc).reshape(-1)[hit] == 10)
    assert np.allclose(rec["allowance"][hit], contrib, rtol=0, atol=1e-12)
    assert np.all(rec["count_slack"][hit] == 1)
    # two margins from the plane: no decision in doubt
    sc = _slab_scene(interpolation=1, clip=[(-1.0, 0.0, 0.0, 2.75 + 4 * eps)])
    rec = oracle.render(sc, lib=lib)
    assert np.all(rec["flags"] == 0) and np.all(rec["allowance"] == 0.0) and np.all(rec["count_slack"] == 0)
    # the margin is a distance: planes with scaled normals flag exactly the same points
    for scale, off, flagged in ((4.0, eps, True), (0.25, 4 * eps, False), (0.25, eps, True), (4.0, 4 * eps, False)):
        sc = _slab_scene(interpolation=1, clip=[(-scale, 0.0, 0.0, scale * (2.75 + off))])
        rec = oracle.render(sc, lib=lib)
        want = 0.9 ** 5 * contrib if flagged else 0.0
        assert np.allclose(rec["allowance"][hit], want, rtol=0, atol=1e-12), (scale, off, rec["allowance"][hit])
        assert np.all(rec["flags"][hit] == (1 if flagged else 0)), (scale, off)
    # box exit: a scan point half a margin before the exit face (kept), and one half a margin past it
    for L, step, n in ((2, 5461 / 4096, 2), (1, 2731 / 4096, 1)):
        sc = _slab_scene(L=L, step=step, interpolation=1)
        rec, hit = oracle.render(sc, lib=lib), _hit_mask(sc).reshape(-1)
        assert abs(1.5 * step - L) == eps
        assert np.all(_cnt(rec, sc).reshape(-1)[hit] == n), (L, np.unique(rec["samples"]))
        assert np.allclose(rec["allowance"][hit], 0.9 * contrib, rtol=0, atol=1e-12), (L, rec["allowance"][hit])
        assert np.all(rec["count_slack"][hit] == 1) and np.all(rec["kinds"][hit] == oracle.oracle.FLAG_EXIT)
    # trilinear sampling of the slab has no decision within a margin at all (the nearest-cell
    # camera of the closed-form pins puts one pixel column on a cell boundary)
    sc = _slab_scene(interpolation=1)
    rec = oracle.render(sc, lib=lib)
    assert np.all(rec["flags"] == 0) and np.all(rec["allowance"] == 0.0)


def pin_allowance_termination(lib):
    a10 = 1.0 - 0.9 ** 10                           # opacity after 10 scan points of alpha 0.1
    a11 = 1.0 - 0.9 ** 11
    for theta, n, flagged in ((a10 + 5e-5, 11, True), (a10 - 5e-5, 10, True),
                              (a10 - 5e-4, 10, False), (a10 + 5e-4, 11, False)):
        sc = _slab_scene(L=40, ert=theta, interpolation=1)
        rec, hit = oracle.render(sc, lib=lib), _hit_mask(sc).reshape(-1)
        assert np.all(_cnt(rec, sc).reshape(-1)[hit] == n), (theta, np.unique(rec["samples"]))
        want = 0.9 ** 10 if flagged else 0.0         # 1 - A at the point next to the threshold
        assert np.allclose(rec["allowance"][hit], want, rtol=0, atol=1e-12), (theta, rec["allowance"][hit])
        assert np.all(rec["flags"][hit] == (1 if flagged else 0))
        assert np.all(rec["count_slack"] == 0)
    assert a11 - (a10 + 5e-4) > 1e-2                 # the unflagged cases stay outside 100x the margin


def pin_allowance_brute_force(lib):
    """The decision bookkeeping against the brute-force loop's own, with margins magnified
    (delta 0.05 and 0.2 voxels, opacity margins 0.05 and 0.02) so that every kind of
    decision occurs many times; and no allowance without a flagged decision."""
    n_flagged = {1: 0, 2: 0, 4: 0, 8: 0}
    for seed in range(24):
        sc = configs.random_small_scene(seed)
        for delta, em in ((0.05, 0.05), (0.2, 0.02)):
            rec = oracle.render(sc, delta=delta, ert_margin=em, lib=lib)
            b = brute.render_flagged(sc, delta, em)
            assert np.array_equal(np.array(b["samples"]).reshape(-1), rec["samples"]), seed
            assert np.array_equal(np.array(b["flags"]).reshape(-1), rec["flags"]), seed
            assert np.array_equal(np.array(b["count_slack"]).reshape(-1), rec["count_slack"]), seed
            assert np.allclose(np.array(b["allowance"]).reshape(-1), rec["allowance"], rtol=0, atol=1e-12), seed
            assert np.all(rec["allowance"][rec["flags"] == 0] == 0.0)
            for k in n_flagged:
                n_flagged[k] += int(((rec["kinds"] & k) != 0).sum())
        # at the real margins the same scenes rarely flag anything, and never allow without a flag
        rec = oracle.render(sc, lib=lib)
        assert np.all(rec["allowance"][rec["flags"] == 0] == 0.0)
        assert np.all(rec["count_slack"] <= rec["flags"])
    assert all(v >= 20 for v in n_flagged.values()), n_flagged


def pin_iso_allowance(lib):
    """Iso mode: a decision within its margin leaves the pixel unconstrained only when it can
    move the crossing; otherwise it moves at most the sample count."""
    eps = 2.0 ** -13
    FREE = 1 << 30

    def centre(rec, sc):
        return rec[(sc.height // 2) * sc.width + sc.width // 2]

    # the crossing half-way between the scan points at 7.25 and 7.75 (values 1/64 from iso)
    sc = _iso_ramp_scene((1.0, 0.0, 0.0), 0.5)
    rec = oracle.render(sc, lib=lib)
    assert np.all(rec["flags"] == 0) and np.all(rec["allowance"] == 0.0) and np.all(rec["count_slack"] == 0)
    # the crossing on a scan point (value 0.515625 at x = 7.75 exactly): either side is right
    sc = _iso_ramp_scene((1.0, 0.0, 0.0), 0.515625)
    rec = oracle.render(sc, lib=lib)
    assert np.all(rec["kinds"] & oracle.oracle.FLAG_ISO) and np.all(rec["allowance"] == 2.0)
    assert np.all(rec["count_slack"] == FREE)
    # the margin of the iso comparison: the value's change over +-delta per axis (0.0625 delta along
    # the ramp) plus 2^-16 of its magnitude: 3.84e-5 at the point x = 7.75 (value 0.515625)
    margin = 0.0625 * _D + 2.0 ** -16 * (1.0 + 0.515625)
    for off, flagged in ((3e-5, True), (-3e-5, True), (1e-4, False), (-1e-4, False)):
        assert (abs(off) < margin) == flagged
        sc = _iso_ramp_scene((1.0, 0.0, 0.0), 0.515625 + off)
        rec = oracle.render(sc, lib=lib)
        assert np.all((rec["flags"] > 0) == flagged), (off, np.unique(rec["flags"]))
        assert np.all(rec["allowance"] == (2.0 if flagged else 0.0)), off
    # a kink: cell values 0.5 + (4 - i) left of cell 4, 0.5 from it on; one scan point (step
    # 9 + 2^-12) half a margin right of cell centre 4.5: the value is 0.5 there and to the right,
    # and rises by 2^-13 over delta to the left, so the margin is the larger, left-hand change
    dims = (8, 3, 3)
    xs = np.arange(-1, 9)
    row = np.where(xs < 4, 0.5 + (4 - xs), 0.5).astype(np.float32)
    kink = make_source("kink", np.broadcast_to(row[None, None, :], (5, 5, 10)).copy(), guard=1,
                       tf=configs.constant_tf((0.5, 0.5, 0.5), 1.0))
    cam = configs.axis_camera(dims, axis=0, width=3, height=3, ortho_height=3.0)
    margin = 2.0 ** -13 + 2.0 ** -16 * 1.5
    for off, flagged in ((0.7 * margin, True), (1.3 * margin, False)):
        kink.iso = 0.5 + off
        sc = Scene(dims=dims, sources=[kink], camera=cam, width=3, height=3, step=9.0 + 2.0 ** -12,
                   interpolation=1, ert_threshold=1.0, mode="iso")
        rec = oracle.render(sc, lib=lib)
        assert np.all(rec["samples"] == 1)
        assert np.all((rec["flags"] > 0) == flagged), (off, rec["flags"])
    base = _iso_ramp_scene((1.0, 0.0, 0.0), 0.5)
    # a plane half a margin from a kept point far in front of the crossing: count +-1 only
    for x0 in (2.25 - eps, 2.25 + eps):
        sc = base.with_(clip=[(1.0, 0.0, 0.0, -x0)])
        c = centre(oracle.render(sc, lib=lib), sc)
        assert c["flags"] == 1 and c["allowance"] == 0.0 and c["count_slack"] == 1, (x0, c)
        assert c["rgba"][3] == 1.0 and c["samples"] == (12 if x0 < 2.25 else 11)
    # the same at the crossing point (kept or dropped): the crossing moves
    for x0 in (7.75 + eps, 7.75 - eps):
        sc = base.with_(clip=[(-1.0, 0.0, 0.0, x0)])
        c = centre(oracle.render(sc, lib=lib), sc)
        assert c["flags"] >= 1 and c["allowance"] == 2.0 and c["count_slack"] == FREE, (x0, c)
    # the point in front of the crossing kept half a margin inside a plane: dropped, the crossing
    # would have no point in front of it on this side of the plane
    sc = base.with_(clip=[(1.0, 0.0, 0.0, -(7.25 - eps))])
    c = centre(oracle.render(sc, lib=lib), sc)
    assert c["rgba"][3] == 1.0 and c["samples"] == 2 and c["allowance"] == 2.0, c
    # a dropped point whose kept value would cross with the next kept one (iso between 2.25 and 2.75)
    sc = _iso_ramp_scene((1.0, 0.0, 0.0), 0.1875).with_(clip=[(1.0, 0.0, 0.0, -(2.25 + eps))])
    c = centre(oracle.render(sc, lib=lib), sc)
    assert c["rgba"][3] == 0.0 and c["allowance"] == 2.0, c
    # two margins away: nothing in doubt
    sc = _iso_ramp_scene((1.0, 0.0, 0.0), 0.1875).with_(clip=[(1.0, 0.0, 0.0, -(2.25 + 4 * eps))])
    c = centre(oracle.render(sc, lib=lib), sc)
    assert c["flags"] == 0 and c["allowance"] == 0.0 and c["count_slack"] == 0, c


# ---------------------------------------------------------------------------
# frame encode: 8-bit quantization of the premultiplied image
# ---------------------------------------------------------------------------

def pin_encode_rgba8(lib):
    from fractions import Fraction
    # every code k is reached exactly at k/255 (rounded to FP32), 0 and 1 at the ends
    k = np.arange(256)
    v = (k / 255.0).astype(np.float32)
    img = np.stack([v, v, v, v], axis=-1)
    q = oracle.encode_rgba8(img, lib=lib)
    assert np.array_equal(q[:, 0], k.astype(np.uint8)) and np.array_equal(q[:, 3], k.astype(np.uint8))
    # out of range and NaN
    odd = np.array([[-1.0, np.nan, 2.0, np.inf], [-np.inf, -0.0, 1e-30, 0.99999994]], dtype=np.float32)
    assert oracle.encode_rgba8(odd, lib=lib).tolist() == [[0, 0, 255, 255], [0, 0, 0, 255]]
    # against exact rational rounding: |q - 255 v| <= 1/2, equality allowed only at a tie of the exact value
    rng = np.random.default_rng(5)
    r = rng.random((4000, 4), dtype=np.float32)
    qr = oracle.encode_rgba8(r, lib=lib).astype(np.int64)
    for x, qq in zip(r.reshape(-1)[:2000], qr.reshape(-1)[:2000]):
        exact = Fraction(float(x)) * 255
        assert abs(Fraction(int(qq)) - exact) <= Fraction(1, 2) + Fraction(1, 1 << 16), (x, qq)
    # monotone in the value
    srt = np.sort(r.reshape(-1))
    qs = oracle.encode_rgba8(np.repeat(srt[:, None], 4, axis=1), lib=lib)[:, 0].astype(int)
    assert np.all(np.diff(qs) >= 0)
    # over a background: an opaque pixel ignores it, a transparent black one shows it, alpha is 255
    bg = (0.25, 0.5, 1.0)
    px = np.array([[0.2, 0.4, 0.6, 1.0], [0.0, 0.0, 0.0, 0.0], [0.1, 0.1, 0.1, 0.5]], dtype=np.float32)
    qb = oracle.encode_rgba8(px, bg, lib=lib)
    assert qb[0].tolist() == [51, 102, 153, 255]
    assert qb[1].tolist() == [64, 128, 255, 255]
    assert qb[2].tolist() == [int(np.floor((0.1 + 0.5 * b) * 255 + 0.5)) for b in bg] + [255]


ALL_PINS = [pin_constant_slab, pin_constant_slab_weight_and_two_sources, pin_mix_saturation,
            pin_constant_slab_ert, pin_constant_slab_clip, pin_linear_ramp, pin_functor_examples,
            pin_chain_render_equivalence, pin_tf_table, pin_classification_lookup, pin_geometry,
            pin_orientation, pin_perspective_symmetry, pin_brute_force, pin_ert_bound,
            pin_fp16_bf16_reads, pin_iso_plane, pin_iso_bilinear,
            pin_iso_sphere, pin_encode_rgba8, pin_allowance_nearest_boundary, pin_allowance_clip_and_exit,
            pin_allowance_termination, pin_allowance_brute_force, pin_iso_allowance]
