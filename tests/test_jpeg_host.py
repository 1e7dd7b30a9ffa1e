"""The library's host-side JPEG tables (csrc/jpeg_tables.cpp) against the JPEG oracle.

The Huffman code-length procedure, the canonical codes, the scaled
quantisation tables, the DCT matrix, the zigzag map and the marker segments
run on the CPU; this test builds that one file with the host compiler behind a
small C shim and compares every result with oracle/jpeg.py, on random symbol
counts, skewed and Fibonacci-like counts (which force the 16-bit length
limit), single-symbol tables and every quality.
"""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import jpeg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1611_09048_amd", "csrc")

SHIM = r"""
#include "jpeg_internal.h"
extern "C" {
void shim_lengths(const uint32_t* f, uint8_t* l) { isaac::jpeg_code_lengths(f, l); }
int shim_canonical(const uint8_t* l, uint32_t* p, uint8_t* b, uint8_t* v) { return isaac::jpeg_canonical(l, p, b, v); }
void shim_tables(int q, int32_t* dct, int32_t* quant, int32_t* zz, int32_t* qinv) {
    isaac::JpegTables t;
    isaac::jpeg_fill_tables(q, &t);
    for (int i = 0; i < 64; ++i) dct[i] = t.dct[i], zz[i] = t.zz[i], quant[i] = t.quant[0][i], quant[64 + i] = t.quant[1][i];
    for (int i = 0; i < 64; ++i) qinv[i] = t.qinv[0][i], qinv[64 + i] = t.qinv[1][i];
}
size_t shim_headers(int w, int h, int q, const uint8_t* bits, const uint8_t* vals, const int* nvals, uint8_t* out) {
    isaac::JpegTables t;
    isaac::jpeg_fill_tables(q, &t);
    uint8_t b[4][16], v[4][256];
    for (int k = 0; k < 4; ++k) {
        for (int i = 0; i < 16; ++i) b[k][i] = bits[k * 16 + i];
        for (int i = 0; i < 256; ++i) v[k][i] = vals[k * 256 + i];
    }
    return isaac::jpeg_headers(w, h, t, b, v, nvals, out);
}
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("jpeg_host")
    shim = d / "shim.cpp"
    shim.write_text(SHIM)
    so = d / "libjpeg_host.so"
    subprocess.run([gxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(shim),
                    os.path.join(CSRC, "jpeg_tables.cpp"), "-o", str(so)], check=True)
    return ctypes.CDLL(str(so))


def lengths(lib, freq):
    f = (ctypes.c_uint32 * 256)(*freq)
    out = (ctypes.c_uint8 * 256)()
    lib.shim_lengths(f, out)
    return list(out)


def test_code_lengths_match_oracle(lib):
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(60):
        k = int(rng.integers(1, 257))
        f = np.zeros(256, np.int64)
        idx = rng.choice(256, size=k, replace=False)
        f[idx] = rng.integers(1, 5000, size=k)
        cases.append(f)
    for _ in range(20):                                    # heavy skew: long codes, the 16-bit limit
        f = np.zeros(256, np.int64)
        k = int(rng.integers(20, 200))
        f[rng.choice(256, size=k, replace=False)] = (2.0 ** rng.uniform(0, 30, size=k)).astype(np.int64) + 1
        cases.append(f)
    fib = [1, 1]
    while len(fib) < 45:
        fib.append(fib[-1] + fib[-2])
    cases.append(np.array(fib[:30] + [0] * 226))
    for sym in (0, 7, 255):
        one = np.zeros(256, np.int64)
        one[sym] = 3
        cases.append(one)
    for f in cases:
        want = jpeg.code_lengths([int(x) for x in f])
        got = lengths(lib, [int(x) for x in f])
        assert got == want


def test_canonical_matches_oracle(lib):
    rng = np.random.default_rng(6)
    for _ in range(30):
        f = [int(x) for x in rng.integers(0, 300, size=256) * (rng.random(256) < 0.4)]
        f[0] += 1
        ln = jpeg.code_lengths(f)
        codes, vals, counts = jpeg.canonical(ln)
        packed = (ctypes.c_uint32 * 256)()
        bits = (ctypes.c_uint8 * 16)()
        v = (ctypes.c_uint8 * 256)()
        n = lib.shim_canonical((ctypes.c_uint8 * 256)(*ln), packed, bits, v)
        assert n == len(vals) and list(v)[:n] == vals and list(bits) == counts
        for sym in range(256):
            if ln[sym]:
                assert packed[sym] == codes[sym][0] | (codes[sym][1] << 16)
            else:
                assert packed[sym] == 0


@pytest.mark.parametrize("quality", [1, 2, 10, 49, 50, 51, 75, 90, 99, 100])
def test_tables_match_oracle(lib, quality):
    dct = (ctypes.c_int32 * 64)()
    quant = (ctypes.c_int32 * 128)()
    zz = (ctypes.c_int32 * 64)()
    qinv = (ctypes.c_int32 * 128)()
    lib.shim_tables(quality, dct, quant, zz, qinv)
    assert np.array_equal(np.array(dct).reshape(8, 8), jpeg.dct_matrix())
    qt = jpeg.scaled_tables(quality)
    assert np.array_equal(np.array(quant[:64]).reshape(8, 8), qt[0])
    assert np.array_equal(np.array(quant[64:]).reshape(8, 8), qt[1])
    order = jpeg.zigzag_order()
    for k, (r, c) in enumerate(order):
        assert zz[r * 8 + c] == k
    # the device quantises by reciprocal multiply: exact for every dividend below 2^12
    # (|f| <= 1024 plus half a divisor), with 24-bit operands and a product below 2^32
    a = np.arange(4096, dtype=np.uint64)
    for q, r in zip(quant, qinv):
        assert 0 < r < (1 << 24) and int(a[-1]) * r < (1 << 32)
        assert np.array_equal((a * np.uint64(r)) >> np.uint64(20), a // np.uint64(q))


@pytest.mark.parametrize("shape,quality", [((1, 1), 100), ((37, 53), 90), ((8, 16), 20)])
def test_headers_match_oracle(lib, shape, quality):
    """The marker segments equal the oracle's stream up to the entropy-coded data."""
    h, w = shape
    rng = np.random.default_rng(h)
    img = rng.integers(0, 256, size=(h, w, 4), dtype=np.uint8)
    stream = jpeg.encode(img, quality)
    # the oracle's own tables for this frame, recomputed from its symbol counts
    blocks, mw, mh = jpeg.coefficient_blocks(img, quality)
    freq = {k: [0] * 256 for k in ("dc0", "ac0", "dc1", "ac1")}
    prev = [0, 0, 0]
    for m in range(blocks.shape[0]):
        for c in range(3):
            for kind, s, _, _ in jpeg.block_symbols(blocks[m, c], prev[c]):
                freq[f"{kind}{0 if c == 0 else 1}"][s] += 1
            prev[c] = int(blocks[m, c, 0])
    bits = (ctypes.c_uint8 * 64)()
    vals = (ctypes.c_uint8 * 1024)()
    nvals = (ctypes.c_int * 4)()
    for k, key in enumerate(("dc0", "ac0", "dc1", "ac1")):
        _, v, counts = jpeg.canonical(jpeg.code_lengths(freq[key]))
        for i, c in enumerate(counts):
            bits[k * 16 + i] = c
        for i, x in enumerate(v):
            vals[k * 256 + i] = x
        nvals[k] = len(v)
    out = (ctypes.c_uint8 * 4096)()
    n = lib.shim_headers(w, h, quality, bits, vals, nvals, out)
    assert bytes(out[:n]) == stream[:n]
    assert stream[n - 14:n - 12] == b"\xff\xda"           # the headers end with the SOS segment
