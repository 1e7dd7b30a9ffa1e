// Baseline JPEG encoding of an RGBA8 frame on the device.
//
// The paper compresses the composited frame to JPEG before it goes to the
// server (Sec. 3.4).  Here every data-parallel step runs on the GPU:
//   1. coef:   one wave per MCU (8x8 pixels, three components): colour
//              conversion, separable integer DCT through LDS, quantisation,
//              zigzag; 64 int16 per block, blocks in scan order (Y, Cb, Cr per MCU);
//   2. hist:   one wave per block, one lane per coefficient: the block's
//              symbols found from a ballot of the nonzero lanes (run = distance
//              to the previous nonzero lane), counted per table in LDS;
//   (host)     Huffman code lengths and codes per table (Annex K.2);
//   3. bits:   the same symbols, priced with the codes: bits per block;
//   4. scan:   exclusive prefix sum of the block bit counts (bit offsets);
//   5. pack:   each wave assembles its block's bits in LDS (lanes OR their
//              codes in at their own offsets, a wave prefix sum of the lane bit
//              counts), stores the interior words and ORs the two boundary words
//              it may share with its neighbours; the last block adds the 1-bit
//              padding to a byte boundary;
//   6. stuff:  count of 0xFF bytes per 16-byte chunk, a prefix sum of the counts,
//              and the copy that inserts a 0x00 after every 0xFF.
// Between the passes the host reads three small values (the symbol counts,
// the total bit count, the stuffed byte count) to build the tables and size
// the buffers; the coded bytes are copied to the host once, behind the headers.

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "isaac_mi355x.h"
#include "jpeg_internal.h"

namespace isaac {

namespace {

constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kScanItems = 4;             // prefix sums: items per thread
constexpr int kScanChunk = kThreads * kScanItems;
constexpr int kStuffBytes = 16;           // bytes per thread in the stuffing passes
constexpr int kBlockWords = 64;           // LDS words per wave in the pack pass (a block needs <= 56)

__device__ inline int category(int v) { return v ? 32 - __clz(v < 0 ? -v : v) : 0; }

// One lane's share of a block's symbols.  Lane 0 codes the DC difference,
// lane k >= 1 with a nonzero coefficient codes its (run, size) symbol behind
// `zrl` ZRL symbols, lane 63 codes EOB when the last coefficient is zero.
struct LaneSym {
    int table;          // 0 DC luma, 1 AC luma, 2 DC chroma, 3 AC chroma; -1: nothing
    int sym;
    int zrl;
    int size;           // extra bits
    uint32_t extra;
};

__device__ inline LaneSym lane_symbol(const int16_t* __restrict__ coef, long long b, bool live, int lane) {
    const int v = live ? coef[b * 64 + lane] : 0;
    const unsigned long long nz = __ballot(v != 0);
    const int chroma = live && (b % 3) != 0;
    LaneSym s{-1, 0, 0, 0, 0u};
    if (!live) return s;
    if (lane == 0) {
        const int prev = b >= 3 ? coef[(b - 3) * 64] : 0;
        const int diff = v - prev;
        s.table = 2 * chroma;
        s.size = category(diff);
        s.sym = s.size;
        s.extra = (uint32_t)(diff >= 0 ? diff : diff + (1 << s.size) - 1);
    } else if (v != 0) {
        const unsigned long long below = nz & ((1ull << lane) - 1ull) & ~1ull;
        const int prev = below ? 63 - __clzll(below) : 0;
        const int run = lane - prev - 1;
        s.table = 2 * chroma + 1;
        s.zrl = run >> 4;
        s.size = category(v);
        s.sym = ((run & 15) << 4) | s.size;
        s.extra = (uint32_t)(v >= 0 ? v : v + (1 << s.size) - 1);
    } else if (lane == 63) {
        s.table = 2 * chroma + 1;
        s.sym = 0x00;                      // EOB
    }
    return s;
}

__device__ inline unsigned wave_sum(unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline unsigned wave_incl_scan(unsigned v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline unsigned long long wave_incl_scan64(unsigned long long v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// ---- 1. coefficients ----

__global__ __launch_bounds__(kThreads) void jpeg_coef_kernel(const uint8_t* __restrict__ rgba, int width, int height,
                                                             int mcu_cols, long long n_mcu,
                                                             const JpegTables* __restrict__ tab,
                                                             int16_t* __restrict__ coef) {
    __shared__ int S[kWaves][3][64];
    __shared__ int T[kWaves][3][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane >> 3, c = lane & 7;
    // per lane: row pass output (y = r, u = c) needs M[c][*]; column pass (v = r, u = c) needs M[r][*]
    int mu[8], mv[8];
    for (int i = 0; i < 8; ++i) mu[i] = tab->dct[c * 8 + i], mv[i] = tab->dct[r * 8 + i];
    const int q0 = tab->quant[0][lane], q1 = tab->quant[1][lane], zz = tab->zz[lane];
    for (long long m0 = (long long)blockIdx.x * kWaves; m0 < n_mcu; m0 += (long long)gridDim.x * kWaves) {
        const long long mcu = m0 + wave;
        const bool live = mcu < n_mcu;
        if (live) {
            const int by = (int)(mcu / mcu_cols), bx = (int)(mcu - (long long)by * mcu_cols);
            const int x = min(bx * 8 + c, width - 1), y = min(by * 8 + r, height - 1);
            const uint32_t p = *reinterpret_cast<const uint32_t*>(rgba + ((size_t)y * width + x) * 4);
            const int R = p & 255, G = (p >> 8) & 255, B = (p >> 16) & 255;
            const int Y = (19595 * R + 38470 * G + 7471 * B + 32768) >> 16;
            const int Cb = ((-11059 * R - 21709 * G + 32768 * B + 32768) >> 16) + 128;
            const int Cr = ((32768 * R - 27439 * G - 5329 * B + 32768) >> 16) + 128;
            S[wave][0][lane] = min(max(Y, 0), 255) - 128;
            S[wave][1][lane] = min(max(Cb, 0), 255) - 128;
            S[wave][2][lane] = min(max(Cr, 0), 255) - 128;
        }
        __syncthreads();
        if (live)
            for (int k = 0; k < 3; ++k) {
                int acc = 0;
                for (int i = 0; i < 8; ++i) acc += mu[i] * S[wave][k][r * 8 + i];
                T[wave][k][lane] = (acc + 512) >> 10;          // two fractional bits kept
            }
        __syncthreads();
        if (live)
            for (int k = 0; k < 3; ++k) {
                int acc = 0;
                for (int i = 0; i < 8; ++i) acc += mv[i] * T[wave][k][i * 8 + c];
                const int f = (acc + 8192) >> 14;
                const int q = k ? q1 : q0;
                const int mag = ((f < 0 ? -f : f) + (q >> 1)) / q;
                coef[(mcu * 3 + k) * 64 + zz] = (int16_t)(f < 0 ? -mag : mag);
            }
        __syncthreads();
    }
}

// ---- 2. symbol counts ----

__global__ __launch_bounds__(kThreads) void jpeg_hist_kernel(const int16_t* __restrict__ coef, long long n_blocks,
                                                             uint32_t* __restrict__ hist) {
    __shared__ uint32_t H[kJpegTableCount * 256];
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads) H[i] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (long long b = (long long)blockIdx.x * kWaves + wave; b - wave < n_blocks;
         b += (long long)gridDim.x * kWaves) {
        const LaneSym s = lane_symbol(coef, b, b < n_blocks, lane);
        if (s.table >= 0) {
            atomicAdd(&H[s.table * 256 + s.sym], 1u);
            if (s.zrl) atomicAdd(&H[s.table * 256 + 0xF0], (unsigned)s.zrl);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads)
        if (H[i]) atomicAdd(&hist[i], H[i]);
}

// ---- 3. bits per block ----

__device__ inline unsigned lane_bits(const LaneSym& s, const uint32_t* C) {
    if (s.table < 0) return 0;
    const uint32_t* t = C + s.table * 256;
    return (unsigned)s.zrl * (t[0xF0] >> 16) + (t[s.sym] >> 16) + (unsigned)s.size;
}

__global__ __launch_bounds__(kThreads) void jpeg_bits_kernel(const int16_t* __restrict__ coef, long long n_blocks,
                                                             const uint32_t* __restrict__ codes,
                                                             uint32_t* __restrict__ bits) {
    __shared__ uint32_t C[kJpegTableCount * 256];
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads) C[i] = codes[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (long long b = (long long)blockIdx.x * kWaves + wave; b - wave < n_blocks;
         b += (long long)gridDim.x * kWaves) {
        const bool live = b < n_blocks;
        const LaneSym s = lane_symbol(coef, b, live, lane);
        const unsigned total = wave_sum(lane_bits(s, C));
        if (live && lane == 0) bits[b] = total;
    }
}

// ---- 4. prefix sums (exclusive, 64-bit) of a uint32 array ----

__device__ inline unsigned long long block_excl_scan(unsigned long long v, unsigned long long* total) {
    __shared__ unsigned long long W[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long incl = wave_incl_scan64(v, lane);
    if (lane == 63) W[wave] = incl;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) before += W[w];
        all += W[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, long long n,
                                                               unsigned long long* __restrict__ part) {
    const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanItems;
    unsigned long long s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    unsigned long long all;
    block_excl_scan(s, &all);
    if (threadIdx.x == 0) part[blockIdx.x] = all;
}

// One workgroup: exclusive scan of the partial sums in place, grand total behind them.
__global__ __launch_bounds__(kThreads) void scan_top_kernel(unsigned long long* __restrict__ part, long long n_parts,
                                                            unsigned long long* __restrict__ total) {
    unsigned long long carry = 0;
    for (long long b0 = 0; b0 < n_parts; b0 += kThreads) {
        const long long i = b0 + threadIdx.x;
        const unsigned long long v = i < n_parts ? part[i] : 0;
        unsigned long long all;
        const unsigned long long ex = block_excl_scan(v, &all);
        if (i < n_parts) part[i] = carry + ex;
        carry += all;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const uint32_t* __restrict__ in, long long n,
                                                              const unsigned long long* __restrict__ part,
                                                              unsigned long long* __restrict__ out) {
    const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    unsigned long long s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        s += v[i];
    }
    unsigned long long all;
    unsigned long long off = part[blockIdx.x] + block_excl_scan(s, &all);
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) {
            out[base + i] = off;
            off += v[i];
        }
}

// ---- 5. bit packing ----

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// OR n (1..27) bits of val, most significant first, in at bit position q of W.
__device__ inline void lds_put(uint32_t* W, int q, uint32_t val, int n) {
    const int w = q >> 5, room = 32 - (q & 31);
    if (n <= room) {
        atomicOr(&W[w], val << (room - n));
    } else {
        const int n2 = n - room;
        atomicOr(&W[w], val >> n2);
        atomicOr(&W[w + 1], val << (32 - n2));
    }
}

__global__ __launch_bounds__(kThreads) void jpeg_pack_kernel(const int16_t* __restrict__ coef, long long n_blocks,
                                                             const uint32_t* __restrict__ codes,
                                                             const unsigned long long* __restrict__ offs,
                                                             uint32_t* __restrict__ words) {
    __shared__ uint32_t C[kJpegTableCount * 256];
    __shared__ uint32_t W[kWaves][kBlockWords];
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads) C[i] = codes[i];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (long long b0 = (long long)blockIdx.x * kWaves; b0 < n_blocks; b0 += (long long)gridDim.x * kWaves) {
        const long long b = b0 + wave;
        const bool live = b < n_blocks;
        W[wave][lane] = 0u;
        __syncthreads();
        const LaneSym s = lane_symbol(coef, b, live, lane);
        const unsigned nb = lane_bits(s, C);
        const unsigned incl = wave_incl_scan(nb, lane);
        const unsigned block_bits = __shfl(incl, 63);
        const unsigned long long p0 = live ? offs[b] : 0ull;
        const int off0 = (int)(p0 & 31);
        int nw = 0;
        if (live) {
            int q = off0 + (int)(incl - nb);
            if (s.table >= 0) {
                const uint32_t* t = C + s.table * 256;
                const uint32_t z = t[0xF0];
                for (int i = 0; i < s.zrl; ++i) {
                    lds_put(W[wave], q, z & 0xFFFFu, (int)(z >> 16));
                    q += (int)(z >> 16);
                }
                const uint32_t e = t[s.sym];
                const int len = (int)(e >> 16);
                lds_put(W[wave], q, ((e & 0xFFFFu) << s.size) | s.extra, len + s.size);
            }
            int end = off0 + (int)block_bits;
            if (b == n_blocks - 1) {
                const int pad = (int)((8 - ((p0 + block_bits) & 7)) & 7);
                if (pad && lane == 0) lds_put(W[wave], end, (1u << pad) - 1u, pad);
                end += pad;
            }
            nw = (end + 31) >> 5;
        }
        __syncthreads();
        if (live && lane < nw) {
            uint32_t* g = words + (p0 >> 5) + lane;
            if (lane == 0 || lane == nw - 1)
                atomicOr(g, W[wave][lane]);   // may be shared with the neighbouring block
            else
                *g = W[wave][lane];
        }
        __syncthreads();
    }
}

// ---- 6. byte stuffing ----

__device__ inline uint32_t stream_byte(const uint32_t* words, unsigned long long k) {
    return (words[k >> 2] >> (24 - 8 * (int)(k & 3))) & 0xFFu;
}

__global__ __launch_bounds__(kThreads) void stuff_count_kernel(const uint32_t* __restrict__ words,
                                                               unsigned long long n_bytes,
                                                               uint32_t* __restrict__ counts, long long n_chunks) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= n_chunks) return;
    const unsigned long long k0 = (unsigned long long)t * kStuffBytes;
    uint32_t n = 0;
    for (int i = 0; i < kStuffBytes; ++i)
        if (k0 + i < n_bytes && stream_byte(words, k0 + i) == 0xFFu) ++n;
    counts[t] = n;
}

__global__ __launch_bounds__(kThreads) void stuff_write_kernel(const uint32_t* __restrict__ words,
                                                               unsigned long long n_bytes,
                                                               const unsigned long long* __restrict__ ff_before,
                                                               long long n_chunks, uint8_t* __restrict__ out) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= n_chunks) return;
    const unsigned long long k0 = (unsigned long long)t * kStuffBytes;
    unsigned long long pos = k0 + ff_before[t];
    for (int i = 0; i < kStuffBytes; ++i) {
        if (k0 + i >= n_bytes) break;
        const uint32_t v = stream_byte(words, k0 + i);
        out[pos++] = (uint8_t)v;
        if (v == 0xFFu) out[pos++] = 0;
    }
}

int grid_for(long long items_per_wave_group, int cap) {
    return (int)std::max(1LL, std::min<long long>(items_per_wave_group, cap));
}

}  // namespace

struct JpegWork {
    JpegTables* tables = nullptr;        // device
    uint32_t* codes = nullptr;           // device [4][256]
    uint32_t* hist = nullptr;            // device [4][256]
    unsigned long long* totals = nullptr;  // device [2]: bit total, 0xFF total
    uint32_t* host_hist = nullptr;       // pinned [4][256]
    unsigned long long* host_totals = nullptr;  // pinned [2]
    uint32_t* host_codes = nullptr;      // pinned [4][256]
    JpegTables host_tables{};
    int quality = -1;
    void* buf[8] = {};
    size_t cap[8] = {};
};

namespace {

enum Buf { B_COEF = 0, B_BITS, B_OFFS, B_PART, B_WORDS, B_CNT, B_FFOFF, B_OUT };

hipError_t grow(JpegWork* w, int i, size_t bytes) {
    if (bytes <= w->cap[i]) return hipSuccess;
    if (w->buf[i]) {
        hipError_t e = hipFree(w->buf[i]);
        w->buf[i] = nullptr;
        w->cap[i] = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&w->buf[i], bytes);
    if (e == hipSuccess) w->cap[i] = bytes;
    return e;
}

// Exclusive prefix sums of n uint32 values into out, total into *total (device).
hipError_t prefix_sum(JpegWork* w, const uint32_t* in, long long n, unsigned long long* out,
                      unsigned long long* total, hipStream_t s) {
    const long long parts = (n + kScanChunk - 1) / kScanChunk;
    hipError_t e = grow(w, B_PART, (size_t)std::max(1LL, parts) * sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    auto* part = static_cast<unsigned long long*>(w->buf[B_PART]);
    scan_reduce_kernel<<<(unsigned)parts, kThreads, 0, s>>>(in, n, part);
    scan_top_kernel<<<1, kThreads, 0, s>>>(part, parts, total);
    scan_apply_kernel<<<(unsigned)parts, kThreads, 0, s>>>(in, n, part, out);
    return hipGetLastError();
}

}  // namespace

JpegWork* jpeg_work_create() { return new JpegWork(); }

void jpeg_work_destroy(JpegWork* w) {
    if (!w) return;
    for (void* p : w->buf)
        if (p) hipFree(p);
    if (w->tables) hipFree(w->tables);
    if (w->codes) hipFree(w->codes);
    if (w->hist) hipFree(w->hist);
    if (w->totals) hipFree(w->totals);
    if (w->host_hist) hipHostFree(w->host_hist);
    if (w->host_totals) hipHostFree(w->host_totals);
    if (w->host_codes) hipHostFree(w->host_codes);
    delete w;
}

int jpeg_encode(JpegWork* w, const uint8_t* rgba8, int width, int height, int quality, void* stream,
                uint8_t* out, size_t capacity, size_t* out_size, char* err, size_t err_len) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto fail = [&](int code, const char* what, hipError_t e) {
        snprintf(err, err_len, "%s%s%s", what, e != hipSuccess ? ": " : "", e != hipSuccess ? hipGetErrorString(e) : "");
        return code;
    };
#define JPEG_TRY(expr)                                                         \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) return fail(ISAAC_ERR_DEVICE, #expr, e_);        \
    } while (0)
    if (!rgba8 || !out_size || width < 1 || height < 1 || width > 65535 || height > 65535)
        return fail(ISAAC_ERR_INVALID_ARGUMENT, "jpeg needs a frame of 1..65535 pixels per side and out_size",
                    hipSuccess);
    if (quality < 1 || quality > 100) return fail(ISAAC_ERR_INVALID_ARGUMENT, "quality must lie in 1..100", hipSuccess);
    const int mcu_cols = (width + 7) / 8, mcu_rows = (height + 7) / 8;
    const long long n_mcu = (long long)mcu_cols * mcu_rows, n_blocks = 3 * n_mcu;
    // symbol counts are 32-bit: at most 64 symbols per block
    if (n_blocks * 64 >= (1LL << 32))
        return fail(ISAAC_ERR_INVALID_ARGUMENT, "frame too large for one JPEG encode", hipSuccess);

    if (!w->tables) {
        JPEG_TRY(hipMalloc(&w->tables, sizeof(JpegTables)));
        JPEG_TRY(hipMalloc(&w->codes, kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipMalloc(&w->hist, kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipMalloc(&w->totals, 2 * sizeof(unsigned long long)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_hist), kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_codes), kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_totals), 2 * sizeof(unsigned long long)));
    }
    if (w->quality != quality) {
        jpeg_fill_tables(quality, &w->host_tables);
        JPEG_TRY(hipMemcpyAsync(w->tables, &w->host_tables, sizeof(JpegTables), hipMemcpyHostToDevice, s));
        JPEG_TRY(hipStreamSynchronize(s));
        w->quality = quality;
    }
    JPEG_TRY(grow(w, B_COEF, (size_t)n_blocks * 64 * sizeof(int16_t)));
    JPEG_TRY(grow(w, B_BITS, (size_t)n_blocks * sizeof(uint32_t)));
    JPEG_TRY(grow(w, B_OFFS, (size_t)n_blocks * sizeof(unsigned long long)));
    auto* coef = static_cast<int16_t*>(w->buf[B_COEF]);
    auto* bits = static_cast<uint32_t*>(w->buf[B_BITS]);
    auto* offs = static_cast<unsigned long long*>(w->buf[B_OFFS]);

    // 1-2: coefficients and symbol counts
    const int groups_mcu = grid_for((n_mcu + kWaves - 1) / kWaves, 2048);
    const int groups_blk = grid_for((n_blocks + kWaves - 1) / kWaves, 2048);
    fill_u32_kernel<<<4, 256, 0, s>>>(w->hist, kJpegTableCount * 256);
    jpeg_coef_kernel<<<groups_mcu, kThreads, 0, s>>>(rgba8, width, height, mcu_cols, n_mcu, w->tables, coef);
    jpeg_hist_kernel<<<std::min(groups_blk, 1024), kThreads, 0, s>>>(coef, n_blocks, w->hist);
    JPEG_TRY(hipGetLastError());
    JPEG_TRY(hipMemcpyAsync(w->host_hist, w->hist, kJpegTableCount * 256 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    JPEG_TRY(hipStreamSynchronize(s));

    // Huffman tables
    uint8_t bitsl[4][16], vals[4][256];
    int nvals[4];
    for (int k = 0; k < kJpegTableCount; ++k) {
        uint8_t len[256];
        jpeg_code_lengths(w->host_hist + k * 256, len);
        nvals[k] = jpeg_canonical(len, w->host_codes + k * 256, bitsl[k], vals[k]);
    }
    JPEG_TRY(hipMemcpyAsync(w->codes, w->host_codes, kJpegTableCount * 256 * sizeof(uint32_t), hipMemcpyHostToDevice, s));

    // 3-4: bit counts and offsets
    jpeg_bits_kernel<<<groups_blk, kThreads, 0, s>>>(coef, n_blocks, w->codes, bits);
    JPEG_TRY(hipGetLastError());
    JPEG_TRY(prefix_sum(w, bits, n_blocks, offs, w->totals, s));
    JPEG_TRY(hipMemcpyAsync(w->host_totals, w->totals, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    JPEG_TRY(hipStreamSynchronize(s));
    const unsigned long long total_bits = w->host_totals[0];
    const unsigned long long n_bytes = (total_bits + 7) / 8;
    const long long n_words = (long long)((n_bytes + 3) / 4) + 1;
    const long long n_chunks = (long long)((n_bytes + kStuffBytes - 1) / kStuffBytes);

    // 5: packing
    JPEG_TRY(grow(w, B_WORDS, (size_t)n_words * sizeof(uint32_t)));
    auto* words = static_cast<uint32_t*>(w->buf[B_WORDS]);
    fill_u32_kernel<<<grid_for((n_words + 255) / 256, 1024), 256, 0, s>>>(words, n_words);
    jpeg_pack_kernel<<<groups_blk, kThreads, 0, s>>>(coef, n_blocks, w->codes, offs, words);
    JPEG_TRY(hipGetLastError());

    // 6: stuffing
    JPEG_TRY(grow(w, B_CNT, (size_t)std::max(1LL, n_chunks) * sizeof(uint32_t)));
    JPEG_TRY(grow(w, B_FFOFF, (size_t)std::max(1LL, n_chunks) * sizeof(unsigned long long)));
    JPEG_TRY(grow(w, B_OUT, (size_t)std::max(1ULL, 2 * n_bytes)));
    auto* cnt = static_cast<uint32_t*>(w->buf[B_CNT]);
    auto* ffoff = static_cast<unsigned long long*>(w->buf[B_FFOFF]);
    auto* dst = static_cast<uint8_t*>(w->buf[B_OUT]);
    const unsigned stuff_groups = (unsigned)((n_chunks + kThreads - 1) / kThreads);
    stuff_count_kernel<<<stuff_groups, kThreads, 0, s>>>(words, n_bytes, cnt, n_chunks);
    JPEG_TRY(hipGetLastError());
    JPEG_TRY(prefix_sum(w, cnt, n_chunks, ffoff, w->totals + 1, s));
    stuff_write_kernel<<<stuff_groups, kThreads, 0, s>>>(words, n_bytes, ffoff, n_chunks, dst);
    JPEG_TRY(hipGetLastError());
    JPEG_TRY(hipMemcpyAsync(w->host_totals + 1, w->totals + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    JPEG_TRY(hipStreamSynchronize(s));
    const size_t coded = (size_t)(n_bytes + w->host_totals[1]);

    uint8_t hdr[kJpegHeaderMax];
    const size_t hdr_len = jpeg_headers(width, height, w->host_tables, bitsl, vals, nvals, hdr);
    const size_t need = hdr_len + coded + 2;
    *out_size = need;
    if (!out || capacity < need)
        return fail(ISAAC_ERR_INVALID_ARGUMENT, "output capacity below the stream size (written to out_size)",
                    hipSuccess);
    memcpy(out, hdr, hdr_len);
    if (coded) JPEG_TRY(hipMemcpyAsync(out + hdr_len, dst, coded, hipMemcpyDeviceToHost, s));
    JPEG_TRY(hipStreamSynchronize(s));
    out[hdr_len + coded] = 0xFF;
    out[hdr_len + coded + 1] = 0xD9;                            // EOI
    return 0;
#undef JPEG_TRY
}

}  // namespace isaac
