"""Pins of the JPEG oracle (oracle/jpeg.py) against what is fixed outside it.

* Pillow's decoder (libjpeg, an independent implementation of the standard)
  must accept every stream and reproduce the frame within the bound the
  quantisation allows; at quality 100 and on a constant frame it is nearly exact;
* the decoded frame must equal, within the rounding of a decoder, this test's
  own reconstruction from the oracle's quantised coefficients (dequantise,
  inverse DCT in float64, inverse JFIF colour), which ties the bit stream to
  the coefficients;
* the integer DCT stays within 0.75 of the exact DCT in float64 (row-pass
  rounding 1/8, 12-bit cosines, column-pass rounding 1/2);
* Huffman code lengths satisfy the Kraft inequality, stay within 16 bits,
  leave the all-ones code unused and are canonical (prefix-free);
* planted mistakes in a copy of the oracle are caught by these pins.
"""

import io
import math
import re

import numpy as np
import pytest

PIL = pytest.importorskip("PIL.Image")

from oracle import jpeg  # noqa: E402


def decode(b: bytes) -> np.ndarray:
    return np.asarray(PIL.open(io.BytesIO(b)).convert("RGB")).astype(np.int64)


def smooth(h, w, seed=0):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:h, 0:w]
    img = np.zeros((h, w, 4), np.uint8)
    for c in range(3):
        a, b, p = rng.uniform(4, 12), rng.uniform(4, 12), rng.uniform(0, 6)
        img[..., c] = np.clip(128 + 90 * np.sin(x / a + p) * np.cos(y / b), 0, 255).astype(np.uint8)
    img[..., 3] = 255
    return img


def reconstruct(mod, rgba8, quality):
    """Frame from the oracle's coefficients: dequantise, exact inverse DCT, inverse JFIF colour."""
    blocks, mw, mh = mod.coefficient_blocks(rgba8, quality)
    qt = mod.scaled_tables(quality)
    zz = mod.zigzag_order()
    k = np.arange(8)
    cu = np.where(k == 0, 1 / math.sqrt(2), 1.0)
    basis = 0.5 * cu[:, None] * np.cos((2 * k[None, :] + 1) * k[:, None] * math.pi / 16)   # [u][x]
    comp = np.zeros((mh * 8, mw * 8, 3))
    for m in range(blocks.shape[0]):
        by, bx = divmod(m, mw)
        for c in range(3):
            f = np.zeros((8, 8))
            for i, (r, col) in enumerate(zz):
                f[r, col] = blocks[m, c, i] * qt[0 if c == 0 else 1][r, col]
            comp[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8, c] = basis.T @ f @ basis + 128
    y, cb, cr = comp[..., 0], comp[..., 1] - 128, comp[..., 2] - 128
    rgb = np.stack([y + 1.402 * cr, y - 0.344136 * cb - 0.714136 * cr, y + 1.772 * cb], axis=-1)
    h, w = rgba8.shape[:2]
    return np.clip(np.rint(rgb), 0, 255)[:h, :w]


def pin_decoder_accepts_and_bounds(mod):
    img = smooth(45, 61)
    for q, min_psnr in ((10, 20.0), (50, 27.0), (90, 35.0), (100, 45.0)):
        d = decode(mod.encode(img, q))
        assert d.shape == (45, 61, 3)
        mse = ((d - img[..., :3]) ** 2).mean()
        psnr = 10 * math.log10(255 ** 2 / max(mse, 1e-12))
        assert psnr >= min_psnr, (q, psnr)
    const = np.zeros((13, 29, 4), np.uint8)
    const[...] = (200, 30, 90, 255)
    d = decode(mod.encode(const, 90))
    assert np.abs(d - const[..., :3]).max() <= 2
    one = np.array([[[10, 250, 30, 0]]], np.uint8)
    assert np.abs(decode(mod.encode(one, 100)) - one[..., :3]).max() <= 3


def pin_stream_matches_coefficients(mod):
    rng = np.random.default_rng(1)
    for h, w, q in ((24, 40, 75), (17, 9, 95), (64, 64, 30)):
        img = smooth(h, w, seed=h)
        img[::5, ::3, :3] = rng.integers(0, 256, size=img[::5, ::3, :3].shape)   # some sharp detail
        d = decode(mod.encode(img, q))
        r = reconstruct(mod, img, q)
        assert np.abs(d - r).max() <= 3, (h, w, q, np.abs(d - r).max())


def pin_noise_and_stuffing(mod):
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, size=(48, 40, 4), dtype=np.uint8)
    b = mod.encode(img, 97)
    seg = b[b.index(b"\xff\xda") + 14:-2]          # entropy-coded segment
    assert b"\xff\x00" in seg
    assert re.search(rb"\xff[^\x00]", seg) is None  # every 0xFF data byte is stuffed
    d = decode(b)
    assert np.abs(d - reconstruct(mod, img, 97)).max() <= 3


def pin_integer_dct(mod):
    rng = np.random.default_rng(3)
    m = mod.dct_matrix()
    k = np.arange(8)
    cu = np.where(k == 0, 1 / math.sqrt(2), 1.0)
    exact_m = 0.5 * cu[:, None] * np.cos((2 * k[None, :] + 1) * k[:, None] * math.pi / 16)
    for _ in range(200):
        s = rng.integers(-128, 128, size=(8, 8))
        f = mod.fdct(s, m)
        exact = exact_m @ s @ exact_m.T
        assert np.abs(f - exact).max() <= 0.75, np.abs(f - exact).max()
    flat = np.full((8, 8), 37)
    f = mod.fdct(flat, m)
    assert f[0, 0] == 37 * 8 and np.count_nonzero(f) == 1


def pin_gray_block_coefficients(mod):
    """A gray frame R = G = B = v has Y = v and Cb = Cr = 128 exactly (the weights sum to
    one), so its luma DC is round(8 (v - 128) / Q00) (half away from zero) and all else is 0."""
    for v, q in ((165, 50), (91, 50), (200, 75), (128, 90)):
        img = np.zeros((8, 16, 4), np.uint8)
        img[..., :3] = v
        blocks, mw, mh = mod.coefficient_blocks(img, q)
        q00 = int(mod.scaled_tables(q)[0][0, 0])
        num = 8 * (v - 128)
        expect = int(math.copysign(math.floor(abs(num) / q00 + 0.5), num)) if num else 0
        assert blocks.shape == (2, 3, 64)
        assert (blocks[:, 0, 0] == expect).all(), (v, q, blocks[:, 0, 0], expect)
        assert not blocks[:, 0, 1:].any() and not blocks[:, 1:].any()


def pin_huffman_lengths(mod):
    rng = np.random.default_rng(4)
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    skew = [2 ** k for k in range(45)] + [0] * 211   # Huffman depth 45 before the 16-bit limit
    cases = [list(rng.integers(0, 1000, size=256)), [0] * 256, fib + [0] * 216, skew]
    cases[1][7] = 5
    for freq in cases:
        lengths = mod.code_lengths(freq)
        used = [v for v in range(256) if freq[v] > 0]
        assert sorted(v for v in range(256) if lengths[v]) == used
        assert max(lengths) <= 16
        kraft = sum(2.0 ** -l for l in lengths if l)
        assert kraft < 1.0                          # the all-ones code stays free
        codes, vals, counts = mod.canonical(lengths)
        words = [format(c, f"0{l}b") for c, l in codes.values()]
        for a in words:
            assert a != "1" * len(a)
            for b in words:
                assert a == b or not b.startswith(a)
        assert sum(counts) == len(used)


ALL = [pin_decoder_accepts_and_bounds, pin_stream_matches_coefficients, pin_noise_and_stuffing, pin_integer_dct,
       pin_gray_block_coefficients, pin_huffman_lengths]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(jpeg)


MUTANTS = [
    ("zigzag_transposed", "        out.extend(cells)", "        out.extend((c, r) for r, c in cells)"),
    ("dc_not_differenced", "    diff = int(coef[0]) - prev_dc", "    diff = int(coef[0])"),
    ("no_stuffing", "            if byte == 0xFF:\n                out.append(0x00)", "            pass"),
    ("cb_sign", "    cb = ((-11059 * r - 21709 * g + 32768 * b + 32768) >> 16) + 128",
     "    cb = ((11059 * r - 21709 * g + 32768 * b + 32768) >> 16) + 128"),
    ("quality_scale", "    scale = 5000 // quality if quality < 50 else 200 - 2 * quality",
     "    scale = 5000 // quality if quality < 50 else 200 - quality"),
    ("dct_transposed", "    return (m @ t + 8192) >> 14", "    return ((m @ t + 8192) >> 14).T"),
    ("negative_extra_bits", "diff if diff >= 0 else diff + (1 << s) - 1", "diff if diff >= 0 else -diff"),
    ("eob_missing", "    if last < 63:\n        syms.append", "    if False:\n        syms.append"),
    ("no_length_limit", "    for i in range(max(size), 16, -1):", "    for i in range(0):"),
    ("reserved_kept", "    bits[i] -= 1\n", "    bits[i] -= 0\n"),
    ("quantize_truncates", "    mag = (np.abs(f) + q // 2) // q", "    mag = np.abs(f) // q"),
]


def _mutant(find, repl):
    import types
    src = open(jpeg.__file__).read()
    assert src.count(find) == 1, find
    mod = types.ModuleType("jpeg_mutant")
    exec(compile(src.replace(find, repl), "jpeg_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, find, repl):
    mod = _mutant(find, repl)
    caught = False
    for pin in ALL:
        try:
            pin(mod)
        except Exception:                       # a failed pin, or a stream the decoder rejects
            caught = True
            break
    assert caught, f"mutant {name} survives every pin"
