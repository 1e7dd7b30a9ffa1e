"""Frame encode on the GPU (RGBA32F -> RGBA8), bit-exact against the oracle.

The 8-bit codes are integer results decided by FP32 arithmetic; both sides
take them in FP32 with every operation rounded separately, so they must agree
exactly on every input, including NaN, infinities, out-of-range values and
exact rounding ties.
"""

import numpy as np
import pytest

import oracle
from parity import log
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


def hard_values(rng, n):
    """Random values plus ties (k + 1/2)/255, codes k/255, their FP32 neighbours and specials."""
    k = np.arange(256, dtype=np.float64)
    ties = ((k + 0.5) / 255.0).astype(np.float32)
    codes = (k / 255.0).astype(np.float32)
    near = np.concatenate([np.nextafter(ties, np.float32(2)), np.nextafter(ties, np.float32(-1)),
                           np.nextafter(codes, np.float32(2)), np.nextafter(codes, np.float32(-1))])
    special = np.array([np.nan, np.inf, -np.inf, -0.0, 0.0, 1.0, -1e-30, 1e-30, 1.0000001, 0.99999994, 3.0],
                       dtype=np.float32)
    rand = rng.random(n, dtype=np.float32) * np.float32(1.2) - np.float32(0.1)
    v = np.concatenate([ties, codes, near, special, rand]).astype(np.float32)
    return v


@pytest.mark.parametrize("background", [None, (0.25, 0.5, 1.0), (0.1, 0.2, 0.3)])
@pytest.mark.parametrize("shape", [(1, 1), (7, 13), (1080, 1920)])
def test_encode_bit_exact(ctx, background, shape):
    import torch
    h, w = shape
    rng = np.random.default_rng(h * 7 + w)
    v = hard_values(rng, h * w * 4)
    img = rng.permutation(v)[: h * w * 4] if v.size >= h * w * 4 else np.resize(rng.permutation(v), h * w * 4)
    img = img.reshape(h, w, 4).astype(np.float32)
    d_img = torch.from_numpy(img).cuda()
    d_out = torch.zeros((h, w, 4), dtype=torch.uint8, device="cuda")
    ctx.encode_rgba8(d_img.data_ptr(), w, h, d_out.data_ptr(), background)
    got = d_out.cpu().numpy()
    want = oracle.encode_rgba8(img, background)
    mism = int((got != want).sum())
    log(f"encode {h}x{w} bg={background}: {mism} mismatching bytes of {got.size}")
    assert mism == 0


def test_served_image_as_rgba8(ctx):
    """isaac_read_image_rgba8 equals the oracle's encode of the served float image."""
    from paper_1611_09048_amd import device
    sc = configs.pic3(n=32, width=120, height=90)
    vol = device.upload_volume(ctx, sc, 3)
    t = ctx.submit(device.render_job(sc, 3, device.new_image(sc)))
    assert t is not None
    f32 = ctx.read_image(t, np.zeros((sc.height, sc.width, 4), dtype=np.float32))
    for bg in (None, (1.0, 1.0, 1.0)):
        q = ctx.read_image_rgba8(t, np.zeros((sc.height, sc.width, 4), dtype=np.uint8), bg)
        assert np.array_equal(q, oracle.encode_rgba8(f32, bg))
    ctx.release(t)
    del vol


def test_encode_rejects_bad_arguments(ctx):
    from paper_1611_09048_amd import binding
    import torch
    a = torch.zeros((2, 2, 4), device="cuda")
    b = torch.zeros((2, 2, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.IsaacError):
        ctx.encode_rgba8(a.data_ptr(), 2, 2, b.data_ptr(), (0.0, 2.0, 0.0))
    with pytest.raises(binding.IsaacError):
        ctx.encode_rgba8(a.data_ptr(), 0, 2, b.data_ptr())


def test_misaligned_pointers_rejected(ctx):
    """Images are accessed a pixel at a time: misaligned device pointers are refused before any launch."""
    import torch
    from paper_1611_09048_amd import binding, device
    a = torch.zeros((4, 4, 4), device="cuda")
    b = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    for rgba, out in ((a.data_ptr() + 4, b.data_ptr()), (a.data_ptr(), b.data_ptr() + 2)):
        with pytest.raises(binding.IsaacError) as e:
            ctx.encode_rgba8(rgba, 2, 2, out)
        assert e.value.code == -1
    with pytest.raises(binding.IsaacError) as e:
        ctx.encode_jpeg(b.data_ptr() + 1, 2, 2, 90)
    assert e.value.code == -1
    sc = configs.pic3(n=16, width=8, height=8)
    vol = device.upload_volume(ctx, sc, 9)
    img = torch.zeros((9, 8, 4), device="cuda")
    with pytest.raises(binding.IsaacError) as e:
        ctx.render([device.render_job(sc, 9, img, out_rgba=img.data_ptr() + 8)])
    assert e.value.code == -1
    with pytest.raises(binding.IsaacError) as e:
        ctx.composite([img.data_ptr() + 4], [img.data_ptr()], 2, 2, img.data_ptr())
    assert e.value.code == -1
    del vol
