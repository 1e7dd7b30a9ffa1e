"""The C ABI's validation rules, each through the library on the GPU: the call
returns the documented error code; a failing isaac_set_sources or
isaac_set_transfer changes nothing (the volume then renders bit for bit as
before: the strong guarantee); a render or served batch holding one invalid
job launches nothing (the valid job's image keeps its fill, no ticket is
issued, serving memory is unchanged) and a later valid render is unchanged.
The rules follow the source, transfer-function and render descriptions of the
paper's interface (Sec. 3.2, 3.3) as the header states them."""

import ctypes
import math

import numpy as np
import pytest

from parity import log
from scenes import configs

pytestmark = pytest.mark.gpu

INVALID, BAD_FUNCTOR, BAD_TRANSFER, NOT_FOUND = -1, -2, -3, -6
VID = 70


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1611_09048_amd import Context, device
    assert torch.cuda.is_available()
    ctx = Context(device=0, mem_budget=256 << 20)
    sc = configs.pic3(n=32, width=64, height=48)
    vol = device.upload_volume(ctx, sc, VID)
    img, cnt = device.new_image(sc), device.new_counts(sc)
    ctx.render([device.render_job(sc, VID, img, cnt)])
    torch.cuda.synchronize()
    ref = (img.cpu().numpy(), cnt.cpu().numpy())
    assert (ref[1] > 0).sum() > 100
    yield ctx, sc, vol, ref
    ctx.close()


def _same_as_before(ctx, sc, ref):
    import torch
    from paper_1611_09048_amd import device
    img, cnt = device.new_image(sc), device.new_counts(sc)
    ctx.render([device.render_job(sc, VID, img, cnt)])
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy(), ref[0]) and np.array_equal(cnt.cpu().numpy(), ref[1])


def _code(fn):
    from paper_1611_09048_amd import IsaacError
    with pytest.raises(IsaacError) as e:
        fn()
    return e.value.code, str(e.value)


def _descs(vol):
    from paper_1611_09048_amd import binding
    return [binding.SourceDesc.from_buffer_copy(d) for d in vol.descs]


def _set(desc, field, value):
    setattr(desc, field, value)
    return desc


SOURCE_CASES = [
    ("f_dim 0", 1, lambda d: _set(d, "f_dim", 0), INVALID),
    ("f_dim 5", 1, lambda d: _set(d, "f_dim", 5), INVALID),
    ("enabled with a NULL component", 1, lambda d: d.comp.__setitem__(1, None) or d, INVALID),
    ("stride not a multiple of the element size", 0, lambda d: d.stride.__setitem__(0, 2) or d, INVALID),
    ("stride whose extent reaches 2 GiB", 0, lambda d: d.stride.__setitem__(2, 1 << 30) or d, INVALID),
    ("misaligned component", 0, lambda d: d.comp.__setitem__(0, d.comp[0] + 2) or d, INVALID),
    ("weight above 1", 2, lambda d: _set(d, "weight", 1.5), INVALID),
    ("weight NaN", 2, lambda d: _set(d, "weight", math.nan), INVALID),
    ("unknown dtype", 0, lambda d: _set(d, "dtype", 7), INVALID),
    ("negative guard", 0, lambda d: _set(d, "guard", -1), INVALID),
    ("chain does not parse", 1, lambda d: _set(d, "functor_chain", b"length | mul(2"), BAD_FUNCTOR),
    ("unknown functor", 1, lambda d: _set(d, "functor_chain", b"lenght"), BAD_FUNCTOR),
    ("argument count outside {1, dim}", 1, lambda d: _set(d, "functor_chain", b"add(1,2)"), BAD_FUNCTOR),
    ("arguments to length", 1, lambda d: _set(d, "functor_chain", b"length(2)"), BAD_FUNCTOR),
    ("more than 8 functors", 0, lambda d: _set(d, "functor_chain", b"|".join([b"mul(2)"] * 9)), BAD_FUNCTOR),
]


@pytest.mark.parametrize("name,src,change,code", SOURCE_CASES, ids=[c[0] for c in SOURCE_CASES])
def test_set_sources_rule_and_strong_guarantee(env, name, src, change, code):
    ctx, sc, vol, ref = env
    descs = _descs(vol)
    descs[src] = change(descs[src])
    got, msg = _code(lambda: ctx.set_sources(VID, sc.dims, descs))
    log(name, "->", got, msg)
    assert got == code, (name, msg)
    _same_as_before(ctx, sc, ref)


def test_set_sources_volume_and_count_rules(env):
    ctx, sc, vol, ref = env
    descs = _descs(vol)
    assert _code(lambda: ctx.set_sources(VID, (0, 32, 32), descs))[0] == INVALID
    assert _code(lambda: ctx.set_sources(VID, (32, 32, (1 << 20) + 1), descs))[0] == INVALID
    assert _code(lambda: ctx.set_sources(VID, sc.dims, descs * 3))[0] == INVALID          # 9 sources
    assert _code(lambda: ctx.set_sources(100000, sc.dims, descs))[0] == NOT_FOUND
    _same_as_before(ctx, sc, ref)


TF_CASES = [
    ("one point", [(0.0, 1, 1, 1, 0.5)]),
    ("not starting at 0", [(0.1, 0, 0, 0, 0), (1.0, 1, 1, 1, 0.1)]),
    ("not ending at 1", [(0.0, 0, 0, 0, 0), (0.9, 1, 1, 1, 0.1)]),
    ("unsorted", [(0.0, 0, 0, 0, 0), (0.6, 1, 0, 0, 0.1), (0.4, 0, 1, 0, 0.1), (1.0, 1, 1, 1, 0.1)]),
    ("repeated x", [(0.0, 0, 0, 0, 0), (0.5, 1, 0, 0, 0.1), (0.5, 0, 1, 0, 0.1), (1.0, 1, 1, 1, 0.1)]),
    ("value above 1", [(0.0, 0, 0, 0, 0), (1.0, 1.2, 1, 1, 0.1)]),
    ("negative value", [(0.0, 0, 0, 0, -0.01), (1.0, 1, 1, 1, 0.1)]),
    ("NaN value", [(0.0, 0, 0, 0, 0), (1.0, 1, math.nan, 1, 0.1)]),
]


@pytest.mark.parametrize("name,points", TF_CASES, ids=[c[0] for c in TF_CASES])
def test_set_transfer_rule_and_strong_guarantee(env, name, points):
    ctx, sc, vol, ref = env
    got, msg = _code(lambda: ctx.set_transfer(VID, 1, points))
    log(name, "->", got, msg)
    assert got == BAD_TRANSFER, (name, msg)
    _same_as_before(ctx, sc, ref)


def _bad_jobs(sc, out):
    """(name, job, expected code): one invalid field each."""
    from paper_1611_09048_amd import binding, device
    mk = lambda **kw: device.render_job(sc, VID, out, **kw)
    cases = []
    j = mk(); j.width = 0; cases.append(("width 0", j, INVALID))
    j = mk(); j.height = -3; cases.append(("negative height", j, INVALID))
    cases.append(("step 0", mk(step=0.0), INVALID))
    cases.append(("negative step", mk(step=-0.5), INVALID))
    cases.append(("NaN step", mk(step=math.nan), INVALID))
    cases.append(("zero clip normal", mk(clip=[(0.0, 0.0, 0.0, 1.0)]), INVALID))
    cases.append(("NaN clip plane", mk(clip=[(1.0, math.nan, 0.0, 1.0)]), INVALID))
    cases.append(("fovy 0", mk(fovy_deg=0.0), INVALID))
    cases.append(("fovy 180", mk(fovy_deg=180.0), INVALID))
    cases.append(("fovy 200", mk(fovy_deg=200.0), INVALID))
    cases.append(("orthographic height 0", mk(projection=binding.ORTHOGRAPHIC, ortho_height=0.0), INVALID))
    cases.append(("unknown projection", mk(projection=5), INVALID))
    cases.append(("unknown interpolation", mk(interpolation=3), INVALID))
    j = mk(clip=[(1.0, 0.0, 0.0, 1.0)]); j.n_clip = 9; cases.append(("9 clip planes", j, INVALID))
    cases.append(("negative threshold", mk(ert_threshold=-0.5), INVALID))
    j = mk(); j.out_rgba = None; cases.append(("no output", j, INVALID))
    j = mk(); j.out_rgba = out.data_ptr() + 4; cases.append(("misaligned output", j, INVALID))
    cases.append(("unknown volume", device.render_job(sc, 999, out), NOT_FOUND))
    cases.append(("weight override above 1", mk(weights=[1.0, 2.0, 1.0]), INVALID))
    cases.append(("transfer handle not live", mk(tf_handles=[4000, 4000, 4000]), NOT_FOUND))
    c = sc.camera
    cases.append(("eye equals center", mk(eye=c.center), INVALID))
    fwd = np.subtract(c.center, c.eye)
    cases.append(("up parallel to the view", mk(up=tuple(fwd)), INVALID))
    cases.append(("up almost parallel to the view", mk(up=tuple(fwd + np.array([1e-9, 0.0, 0.0]))), INVALID))
    return cases


def test_render_rules_all_or_nothing(env):
    """Every invalid job alone, and behind a valid one in the same call: the error code,
    nothing written to the valid job's image, nothing changed for a later render."""
    import torch
    from paper_1611_09048_amd import device
    ctx, sc, vol, ref = env
    scratch = device.new_image(sc)
    names = []
    for name, bad, code in _bad_jobs(sc, scratch):
        got, msg = _code(lambda: ctx.render([bad]))
        assert got == code, (name, msg)
        good_img = torch.full((sc.height, sc.width, 4), 7.0, device="cuda")
        good = device.render_job(sc, VID, good_img)
        got2, _ = _code(lambda: ctx.render([good, bad]))
        assert got2 == code, name
        got3, _ = _code(lambda: ctx.render_noalloc([good, bad]))
        assert got3 == code, name
        torch.cuda.synchronize()
        assert bool((good_img == 7.0).all()), f"{name}: a batch with an invalid job launched"
        names.append(name)
    log("render rules checked:", names)
    _same_as_before(ctx, sc, ref)


def test_served_batch_all_or_nothing(env):
    import torch
    from paper_1611_09048_amd import device
    ctx, sc, vol, ref = env
    before = ctx.serving_usage()
    out = device.new_image(sc)
    for name, bad, code in _bad_jobs(sc, out):
        if name in ("no output", "misaligned output"):
            continue                      # served jobs write to library-owned images
        good = device.render_job(sc, VID, out)
        got, msg = _code(lambda: ctx.submit_batch([good, bad]))
        assert got == code, (name, msg)
        assert ctx.serving_usage() == before, name
    torch.cuda.synchronize()
    t = ctx.submit(device.render_job(sc, VID, out))
    img = np.empty((sc.height, sc.width, 4), np.float32)
    ctx.read_image(t, img)
    ctx.release(t)
    assert np.array_equal(img, ref[0])
    assert ctx.serving_usage()[0] == before[0]
