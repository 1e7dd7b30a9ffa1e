// Host-side tables of the baseline JPEG encoder: quantisation and DCT
// matrices, per-frame Huffman code lengths and codes, and the marker
// segments in front of the entropy-coded data.

#include <math.h>
#include <string.h>

#include <algorithm>

#include "jpeg_internal.h"

namespace isaac {

namespace {

// Example quantisation tables of the JPEG standard, Annex K (Tables K.1 and
// K.2), natural row-major order.
const uint8_t kLuma[64] = {
    16, 11, 10, 16, 24,  40,  51,  61,  12, 12, 14, 19, 26,  58,  60,  55,
    14, 13, 16, 24, 40,  57,  69,  56,  14, 17, 22, 29, 51,  87,  80,  62,
    18, 22, 37, 56, 68,  109, 103, 77,  24, 35, 55, 64, 81,  104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
const uint8_t kChroma[64] = {
    17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
    24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99};

void put16(uint8_t*& p, unsigned v) {
    *p++ = (uint8_t)(v >> 8);
    *p++ = (uint8_t)v;
}

}  // namespace

void jpeg_fill_tables(int quality, JpegTables* t) {
    // zigzag: walk the anti-diagonals u + v = d, upwards (v falling) on even d
    int k = 0;
    for (int d = 0; d < 15; ++d) {
        for (int i = 0; i < 8; ++i) {
            const int v = (d & 1) ? i : d - i;
            const int u = d - v;
            if (v < 0 || v > 7 || u < 0 || u > 7) continue;
            t->zz[v * 8 + u] = k++;
        }
    }
    // quality scaling in percent: 5000/q below 50, 200 - 2q above
    const int scale = quality < 50 ? 5000 / quality : 200 - 2 * quality;
    for (int i = 0; i < 64; ++i) {
        t->quant[0][i] = std::min(255, std::max(1, (kLuma[i] * scale + 50) / 100));
        t->quant[1][i] = std::min(255, std::max(1, (kChroma[i] * scale + 50) / 100));
        for (int c = 0; c < 2; ++c) t->qinv[c][i] = ((1 << 20) + t->quant[c][i] - 1) / t->quant[c][i];
    }
    const double pi = 3.14159265358979323846;
    for (int u = 0; u < 8; ++u)
        for (int x = 0; x < 8; ++x) {
            const double cu = u == 0 ? sqrt(0.5) : 1.0;
            t->dct[u * 8 + x] = (int32_t)floor(4096.0 * 0.5 * cu * cos((2 * x + 1) * u * pi / 16.0) + 0.5);
        }
}

void jpeg_code_lengths(const uint32_t* freq256, uint8_t* len256) {
    // Annex K.2: repeatedly merge the two least frequent entries (ties to the
    // larger symbol value; the merged entry keeps the first one's value), a
    // symbol's code size being the number of merges its subtree takes part in;
    // entry 256 has count 1 and reserves the all-ones code.  The two least
    // entries come from a heap ordered by (count, -value), so a frame's tables
    // take O(n log n) instead of a scan of all entries per merge.
    constexpr int N = 257;
    struct Entry {
        uint64_t f;
        int v, node;
    };
    auto later = [](const Entry& a, const Entry& b) { return a.f != b.f ? a.f > b.f : a.v < b.v; };
    Entry heap[N];
    int n_heap = 0;
    int parent[2 * N];
    for (int v = 0; v < N; ++v) {
        const uint64_t f = v < 256 ? freq256[v] : 1;
        parent[v] = -1;
        if (f) heap[n_heap++] = Entry{f, v, v};
    }
    std::make_heap(heap, heap + n_heap, later);
    int next_node = N;
    while (n_heap > 1) {
        std::pop_heap(heap, heap + n_heap, later);
        const Entry a = heap[--n_heap];
        std::pop_heap(heap, heap + n_heap, later);
        const Entry b = heap[--n_heap];
        const int p = next_node++;
        parent[p] = -1;
        parent[a.node] = p;
        parent[b.node] = p;
        heap[n_heap++] = Entry{a.f + b.f, a.v, p};
        std::push_heap(heap, heap + n_heap, later);
    }
    int size[N];
    for (int v = 0; v < N; ++v) {
        int d = 0;
        for (int q = parent[v]; q >= 0; q = parent[q]) ++d;
        size[v] = d;
    }
    int count[N + 1] = {0};
    int deepest = 0;
    for (int v = 0; v < N; ++v)
        if (size[v]) ++count[size[v]], deepest = std::max(deepest, size[v]);
    // Annex K.3: lengths beyond 16 bits: a pair at the deepest level leaves it,
    // one of them hangs under the longest shorter code, which moves down a level
    for (int i = deepest; i > 16; --i)
        while (count[i] > 0) {
            int j = i - 2;
            while (count[j] == 0) --j;
            count[i] -= 2;
            count[i - 1] += 1;
            count[j + 1] += 2;
            count[j] -= 1;
        }
    int longest = 16;
    while (count[longest] == 0) --longest;
    --count[longest];                          // the reserved entry's code
    // lengths back to the symbols in order of (merge depth, value): a counting sort by depth
    int per_depth[N + 1] = {0};
    for (int v = 0; v < 256; ++v)
        if (size[v]) ++per_depth[size[v]];
    int first[N + 1];
    first[0] = 0;
    for (int d = 1; d <= N; ++d) first[d] = first[d - 1] + per_depth[d - 1];
    int order[256];
    for (int v = 0; v < 256; ++v)
        if (size[v]) order[first[size[v]]++] = v;
    memset(len256, 0, 256);
    int k = 0;
    for (int l = 1; l <= 16; ++l)
        for (int c = 0; c < count[l]; ++c) len256[order[k++]] = (uint8_t)l;
}

int jpeg_canonical(const uint8_t* len256, uint32_t* packed256, uint8_t* bits16, uint8_t* vals256) {
    // symbols by (length, value): a counting sort by length
    int per_len[17] = {0};
    for (int v = 0; v < 256; ++v) ++per_len[len256[v]];
    int first[17];
    first[1] = 0;
    for (int l = 2; l <= 16; ++l) first[l] = first[l - 1] + per_len[l - 1];
    const int n = first[16] + per_len[16];
    for (int l = 1; l <= 16; ++l) bits16[l - 1] = (uint8_t)per_len[l];
    for (int v = 0; v < 256; ++v)
        if (len256[v]) vals256[first[len256[v]]++] = (uint8_t)v;
    memset(packed256, 0, 256 * sizeof(uint32_t));
    uint32_t code = 0;
    int l = n ? len256[vals256[0]] : 0;
    for (int i = 0; i < n; ++i) {
        const int li = len256[vals256[i]];
        code <<= (li - l);
        l = li;
        packed256[vals256[i]] = code | ((uint32_t)li << 16);
        ++code;
    }
    return n;
}

size_t jpeg_headers(int width, int height, const JpegTables& t, const uint8_t bits[4][16],
                    const uint8_t vals[4][256], const int nvals[4], uint8_t* out) {
    uint8_t* p = out;
    *p++ = 0xFF, *p++ = 0xD8;                                   // SOI
    *p++ = 0xFF, *p++ = 0xE0;                                   // APP0, JFIF 1.01, aspect 1:1
    put16(p, 16);
    memcpy(p, "JFIF", 5), p += 5;
    *p++ = 1, *p++ = 1, *p++ = 0;
    put16(p, 1), put16(p, 1);
    *p++ = 0, *p++ = 0;
    *p++ = 0xFF, *p++ = 0xDB;                                   // DQT, both tables, zigzag order
    put16(p, 2 + 2 * 65);
    for (int q = 0; q < 2; ++q) {
        *p++ = (uint8_t)q;
        uint8_t zz[64];
        for (int i = 0; i < 64; ++i) zz[t.zz[i]] = (uint8_t)t.quant[q][i];
        memcpy(p, zz, 64), p += 64;
    }
    *p++ = 0xFF, *p++ = 0xC0;                                   // SOF0: 8 bit, 3 components, 1x1
    put16(p, 17);
    *p++ = 8;
    put16(p, (unsigned)height), put16(p, (unsigned)width);
    *p++ = 3;
    const uint8_t comps[9] = {1, 0x11, 0, 2, 0x11, 1, 3, 0x11, 1};
    memcpy(p, comps, 9), p += 9;
    *p++ = 0xFF, *p++ = 0xC4;                                   // DHT, four tables
    size_t dht = 2;
    for (int k = 0; k < 4; ++k) dht += 17 + nvals[k];
    put16(p, (unsigned)dht);
    const uint8_t ids[4] = {0x00, 0x10, 0x01, 0x11};            // class << 4 | destination
    for (int k = 0; k < 4; ++k) {
        *p++ = ids[k];
        memcpy(p, bits[k], 16), p += 16;
        memcpy(p, vals[k], (size_t)nvals[k]), p += nvals[k];
    }
    *p++ = 0xFF, *p++ = 0xDA;                                   // SOS: all components, 0..63
    put16(p, 12);
    const uint8_t sos[10] = {3, 1, 0x00, 2, 0x11, 3, 0x11, 0, 63, 0};
    memcpy(p, sos, 10), p += 10;
    return (size_t)(p - out);
}

}  // namespace isaac
