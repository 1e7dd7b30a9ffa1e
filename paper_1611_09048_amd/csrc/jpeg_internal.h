// Library-private interface of the baseline JPEG encoder (jpeg.hip for the
// device passes, jpeg_tables.cpp for the host-side tables and headers).
//
// The stream is baseline sequential JPEG: JFIF YCbCr, no subsampling, the
// example quantisation tables of the standard (Annex K) scaled by a quality,
// and Huffman tables built per frame from the frame's own symbol counts
// (Annex K.2), so the entropy-coded segment is the shortest those tables allow.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace isaac {

// What the coefficient pass needs, in device memory.
struct JpegTables {
    int32_t dct[64];        // M[u][x] = C(u)/2 cos((2x+1) u pi/16), 12 fractional bits, row u
    int32_t quant[2][64];   // luma, chroma divisors, natural (row-major v, u) order
    int32_t qinv[2][64];    // ceil(2^20 / quant): floor(a / q) = (a * qinv) >> 20 for 0 <= a < 4096
    int32_t zz[64];         // natural index v*8+u -> zigzag position
};

// Huffman code of every symbol of the four tables, index table*256 + symbol,
// tables in the order DC luma, AC luma, DC chroma, AC chroma: code in bits
// 0..15, length in bits 16..23 (0: symbol unused).
constexpr int kJpegTableCount = 4;

// Host side (jpeg_tables.cpp).
void jpeg_fill_tables(int quality, JpegTables* t);
// Code lengths of one table from its symbol counts (Annex K.2 and K.3), 0 for
// an unused symbol; every length lies in 1..16 and the all-ones code stays free.
void jpeg_code_lengths(const uint32_t* freq256, uint8_t* len256);
// Canonical codes from the lengths (Annex C): packed code|length<<16 per
// symbol; bits[16] counts per length and vals[] the symbols by length then
// value (the BITS and HUFFVAL lists of a DHT segment); returns the count of vals.
int jpeg_canonical(const uint8_t* len256, uint32_t* packed256, uint8_t* bits16, uint8_t* vals256);
// Markers SOI..SOS of a frame; returns their byte count (at most kJpegHeaderMax).
constexpr size_t kJpegHeaderMax = 2 + 18 + 134 + 19 + 4 * (17 + 256) + 4 + 14;
size_t jpeg_headers(int width, int height, const JpegTables& t, const uint8_t bits[4][16],
                    const uint8_t vals[4][256], const int nvals[4], uint8_t* out);

// Device side (jpeg.hip).  Scratch buffers owned by the caller's context.
struct JpegWork;
JpegWork* jpeg_work_create();
void jpeg_work_destroy(JpegWork* w);
// Encode an RGBA8 frame (device, rows top to bottom, 4 bytes per pixel, alpha
// ignored) into out (host).  Returns 0, or a negative isaac_status with a
// message in err; on a too small capacity *out_size still receives the size.
int jpeg_encode(JpegWork* w, const uint8_t* rgba8, int width, int height, int quality, void* stream,
                uint8_t* out, size_t capacity, size_t* out_size, char* err, size_t err_len);

}  // namespace isaac
