"""Baseline JPEG encoding of an RGBA8 frame: the reference the device encoder is checked against.

TEST INFRASTRUCTURE ONLY: used by tests/ and nowhere in the library.

The paper compresses the composited image to JPEG on the root rank before
sending it to the server (Sec. 3.6).  It gives no encoder details, so the
encoder is defined here (readings recorded with the design notes) in plain
integer arithmetic, so that every coefficient and every bit is a fixed
function of the input:

* colour: JFIF YCbCr from 8-bit R, G, B with 16-bit fixed-point weights,
  each product sum rounded half up by an arithmetic shift; no subsampling
  (every component 8x8 per MCU);
* samples minus 128, 8x8 blocks in raster order, the frame extended by
  repeating its last column and row;
* forward DCT F = M s M^T with M[u][x] = C(u)/2 cos((2x+1) u pi / 16)
  (C(0) = 1/sqrt(2), else 1), M rounded to 12 fractional bits; the row pass
  keeps 2 fractional bits (rounded half up by a shift of 10), the column pass
  rounds half up by a shift of 14;
* quantisation by the example tables of the JPEG standard (Annex K) scaled
  by a quality 1..100 (5000/q below 50, else 200 - 2q, percent, rounded,
  clamped to 1..255), quotient rounded half away from zero;
* coefficients in zigzag order; DC coded as the difference to the previous
  block of the same component; AC as (run, size) symbols with ZRL and EOB;
* per-frame Huffman tables from the frame's symbol counts (four tables: DC
  and AC for luma and for chroma), built by the code-size procedure of the
  JPEG standard (Annex K.2: repeatedly join the two least frequent entries,
  ties to the larger symbol value, a reserved symbol keeping the all-ones
  code free, lengths limited to 16), codes canonical in order of length then
  symbol value;
* entropy-coded bits MSB first, the last byte padded with 1 bits, 0x00
  stuffed after every 0xFF byte; markers SOI, APP0 (JFIF 1.01), DQT, SOF0,
  DHT, SOS, EOI.
"""

from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

# JPEG standard, Annex K, Tables K.1 and K.2 (natural row-major order)
LUMA_Q = np.array([
    16, 11, 10, 16, 24, 40, 51, 61,
    12, 12, 14, 19, 26, 58, 60, 55,
    14, 13, 16, 24, 40, 57, 69, 56,
    14, 17, 22, 29, 51, 87, 80, 62,
    18, 22, 37, 56, 68, 109, 103, 77,
    24, 35, 55, 64, 81, 104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101,
    72, 92, 95, 98, 112, 100, 103, 99], dtype=np.int64).reshape(8, 8)
CHROMA_Q = np.full((8, 8), 99, dtype=np.int64)
CHROMA_Q[:4, :4] = np.array([[17, 18, 24, 47], [18, 21, 26, 66], [24, 26, 56, 99], [47, 66, 99, 99]])


def zigzag_order() -> List[Tuple[int, int]]:
    """(row, column) of the k-th coefficient in zigzag order: anti-diagonals, alternating direction."""
    out = []
    for d in range(15):
        cells = [(r, d - r) for r in range(8) if 0 <= d - r < 8]
        if d % 2 == 0:
            cells = cells[::-1]           # even diagonals run up and to the right
        out.extend(cells)
    return out


def scaled_tables(quality: int):
    if not 1 <= quality <= 100:
        raise ValueError("quality must lie in 1..100")
    scale = 5000 // quality if quality < 50 else 200 - 2 * quality
    out = []
    for base in (LUMA_Q, CHROMA_Q):
        q = (base * scale + 50) // 100
        out.append(np.clip(q, 1, 255))
    return out


def dct_matrix() -> np.ndarray:
    """M[u][x] = C(u)/2 cos((2x+1) u pi / 16) rounded to 12 fractional bits."""
    m = np.zeros((8, 8), dtype=np.int64)
    for u in range(8):
        cu = 1.0 / math.sqrt(2.0) if u == 0 else 1.0
        for x in range(8):
            m[u, x] = int(math.floor(4096.0 * 0.5 * cu * math.cos((2 * x + 1) * u * math.pi / 16.0) + 0.5))
    return m


def ycbcr(rgb: np.ndarray) -> np.ndarray:
    """(..., 3) uint8 -> (..., 3) int64 Y, Cb, Cr in 0..255 (JFIF weights in 16-bit fixed point)."""
    r, g, b = (rgb[..., i].astype(np.int64) for i in range(3))
    y = (19595 * r + 38470 * g + 7471 * b + 32768) >> 16
    cb = ((-11059 * r - 21709 * g + 32768 * b + 32768) >> 16) + 128
    cr = ((32768 * r - 27439 * g - 5329 * b + 32768) >> 16) + 128
    return np.clip(np.stack([y, cb, cr], axis=-1), 0, 255)


def fdct(block: np.ndarray, m: np.ndarray) -> np.ndarray:
    """8x8 int samples (row = y, column = x) -> coefficients F[v][u] (row = v vertical frequency)."""
    t = (block @ m.T + 512) >> 10             # rows: T[y][u] = sum_x M[u][x] s[y][x], 2 fraction bits kept
    return (m @ t + 8192) >> 14               # columns: F[v][u] = sum_y M[v][y] T[y][u]


def quantize(f: np.ndarray, q: np.ndarray) -> np.ndarray:
    mag = (np.abs(f) + q // 2) // q
    return np.where(f < 0, -mag, mag)


def coefficient_blocks(rgba8: np.ndarray, quality: int) -> Tuple[np.ndarray, int, int]:
    """(MCUs, 3 components, 64 zigzag coefficients), MCU columns, MCU rows."""
    h, w = rgba8.shape[:2]
    mw, mh = (w + 7) // 8, (h + 7) // 8
    ys = np.minimum(np.arange(mh * 8), h - 1)
    xs = np.minimum(np.arange(mw * 8), w - 1)
    padded = rgba8[ys][:, xs, :3]
    comp = ycbcr(padded) - 128
    m = dct_matrix()
    qt = scaled_tables(quality)
    zz = zigzag_order()
    zr = np.array([r for r, _ in zz])
    zc = np.array([c for _, c in zz])
    out = np.zeros((mh * mw, 3, 64), dtype=np.int64)
    for by in range(mh):
        for bx in range(mw):
            for c in range(3):
                blk = comp[by * 8:(by + 1) * 8, bx * 8:(bx + 1) * 8, c]
                f = quantize(fdct(blk, m), qt[0 if c == 0 else 1])
                out[by * mw + bx, c] = f[zr, zc]
    return out, mw, mh


def category(v: int) -> int:
    """Number of bits of |v| (0 for 0)."""
    return int(abs(int(v))).bit_length()


def block_symbols(coef: np.ndarray, prev_dc: int):
    """[(table kind 'dc'|'ac', symbol, extra bits value, extra bit count)] of one block."""
    syms = []
    diff = int(coef[0]) - prev_dc
    s = category(diff)
    syms.append(("dc", s, diff if diff >= 0 else diff + (1 << s) - 1, s))
    run = 0
    last = 0
    for k in range(63, 0, -1):
        if coef[k] != 0:
            last = k
            break
    for k in range(1, last + 1):
        v = int(coef[k])
        if v == 0:
            run += 1
            continue
        while run >= 16:
            syms.append(("ac", 0xF0, 0, 0))
            run -= 16
        s = category(v)
        syms.append(("ac", (run << 4) | s, v if v >= 0 else v + (1 << s) - 1, s))
        run = 0
    if last < 63:
        syms.append(("ac", 0x00, 0, 0))
    return syms


def code_lengths(freq: List[int]) -> List[int]:
    """Huffman code length per symbol 0..255 (0: unused), Annex K.2 procedure, limited to 16."""
    f = list(freq[:256]) + [1]                 # symbol 256 reserves the all-ones code
    size = [0] * 257
    others = [-1] * 257
    while True:
        c1 = -1
        for v in range(257):
            if f[v] > 0 and (c1 < 0 or f[v] <= f[c1]):
                c1 = v
        c2 = -1
        for v in range(257):
            if v != c1 and f[v] > 0 and (c2 < 0 or f[v] <= f[c2]):
                c2 = v
        if c2 < 0:
            break
        f[c1] += f[c2]
        f[c2] = 0
        size[c1] += 1
        while others[c1] >= 0:
            c1 = others[c1]
            size[c1] += 1
        others[c1] = c2
        size[c2] += 1
        while others[c2] >= 0:
            c2 = others[c2]
            size[c2] += 1
    bits = [0] * 258                           # a depth can exceed 32 for very skewed counts
    for v in range(257):
        if size[v]:
            bits[size[v]] += 1
    # limit to 16 bits: move pairs of the longest codes up
    for i in range(max(size), 16, -1):
        while bits[i] > 0:
            j = i - 2
            while bits[j] == 0:
                j -= 1
            bits[i] -= 2
            bits[i - 1] += 1
            bits[j + 1] += 2
            bits[j] -= 1
    # drop the reserved symbol's code (the longest)
    i = 16
    while bits[i] == 0:
        i -= 1
    bits[i] -= 1
    # give the lengths back to the symbols: by original size, ties by symbol value
    order = sorted((v for v in range(256) if size[v]), key=lambda v: (size[v], v))
    lengths = [0] * 256
    k = 0
    for length in range(1, 17):
        for _ in range(bits[length]):
            lengths[order[k]] = length
            k += 1
    return lengths


def canonical(lengths: List[int]):
    """{symbol: (code, length)}, HUFFVAL order, BITS counts."""
    vals = sorted((v for v in range(256) if lengths[v]), key=lambda v: (lengths[v], v))
    codes = {}
    code = 0
    prev = 0
    for v in vals:
        code <<= lengths[v] - prev
        prev = lengths[v]
        codes[v] = (code, lengths[v])
        code += 1
    counts = [sum(1 for v in vals if lengths[v] == n) for n in range(1, 17)]
    return codes, vals, counts


def encode(rgba8: np.ndarray, quality: int = 90) -> bytes:
    """JPEG bytes of an (H, W, 4) uint8 frame (alpha ignored)."""
    rgba8 = np.asarray(rgba8, dtype=np.uint8)
    h, w = rgba8.shape[:2]
    if h < 1 or w < 1 or h > 65535 or w > 65535:
        raise ValueError("frame size outside 1..65535")
    blocks, mw, mh = coefficient_blocks(rgba8, quality)
    # symbols, DC predicted per component in MCU order
    syms = []
    prev = [0, 0, 0]
    for mcu in range(blocks.shape[0]):
        row = []
        for c in range(3):
            row.append(block_symbols(blocks[mcu, c], prev[c]))
            prev[c] = int(blocks[mcu, c, 0])
        syms.append(row)
    freq = {k: [0] * 256 for k in ("dc0", "ac0", "dc1", "ac1")}
    for row in syms:
        for c, bs in enumerate(row):
            for kind, s, _, _ in bs:
                freq[f"{kind}{0 if c == 0 else 1}"][s] += 1
    tables = {k: canonical(code_lengths(v)) for k, v in freq.items()}
    # entropy-coded segment
    acc = 0
    nbits = 0
    out = bytearray()

    def put(value: int, n: int):
        nonlocal acc, nbits
        acc = (acc << n) | (value & ((1 << n) - 1))
        nbits += n
        while nbits >= 8:
            byte = (acc >> (nbits - 8)) & 0xFF
            out.append(byte)
            if byte == 0xFF:
                out.append(0x00)
            nbits -= 8
        acc &= (1 << nbits) - 1

    for row in syms:
        for c, bs in enumerate(row):
            for kind, s, extra, n in bs:
                code, length = tables[f"{kind}{0 if c == 0 else 1}"][0][s]
                put(code, length)
                if n:
                    put(extra, n)
    if nbits:
        put((1 << (8 - nbits)) - 1, 8 - nbits)
    # markers
    qt = scaled_tables(quality)
    zz = zigzag_order()
    hdr = bytearray(b"\xff\xd8")
    hdr += b"\xff\xe0" + (16).to_bytes(2, "big") + b"JFIF\x00\x01\x01\x00" + (1).to_bytes(2, "big") \
        + (1).to_bytes(2, "big") + b"\x00\x00"
    dqt = bytearray()
    for t, q in enumerate(qt):
        dqt.append(t)
        dqt += bytes(int(q[r, c]) for r, c in zz)
    hdr += b"\xff\xdb" + (2 + len(dqt)).to_bytes(2, "big") + dqt
    sof = bytearray([8]) + h.to_bytes(2, "big") + w.to_bytes(2, "big") + bytes([3, 1, 0x11, 0, 2, 0x11, 1, 3, 0x11, 1])
    hdr += b"\xff\xc0" + (2 + len(sof)).to_bytes(2, "big") + sof
    dht = bytearray()
    for key, cls_id in (("dc0", 0x00), ("ac0", 0x10), ("dc1", 0x01), ("ac1", 0x11)):
        _, vals, counts = tables[key]
        dht.append(cls_id)
        dht += bytes(counts)
        dht += bytes(vals)
    hdr += b"\xff\xc4" + (2 + len(dht)).to_bytes(2, "big") + dht
    sos = bytearray([3, 1, 0x00, 2, 0x11, 3, 0x11, 0, 63, 0])
    hdr += b"\xff\xda" + (2 + len(sos)).to_bytes(2, "big") + sos
    return bytes(hdr + out + b"\xff\xd9")
