// Baseline JPEG encoding of an RGBA8 frame on the device.
//
// The paper compresses the composited frame to JPEG before it goes to the
// server (Sec. 3.6).  Here every data-parallel step runs on the GPU:
//   1. coef:   one wave per MCU (8x8 pixels, three components): colour
//              conversion, separable integer DCT through LDS, quantisation,
//              zigzag; 64 int16 per block, blocks in scan order (Y, Cb, Cr per MCU);
//   2. hist:   one lane per coefficient, 4 blocks per wave with their loads in
//              flight together: each block's symbols come from a ballot of the
//              nonzero lanes (run = distance to the highest nonzero lane below),
//              counted per table in LDS;
//   (host)     Huffman code lengths and codes per table (Annex K.2);
//   3. bits:   the same symbols priced with the codes: bits per block and per
//              workgroup (16 blocks);
//   4. scan:   one workgroup turns the workgroup bit counts into bit offsets;
//   5. pack:   each workgroup ORs its 16 blocks' codes into an LDS image of its
//              bit range (lane offsets from a wave prefix sum), stores the words
//              it owns alone and ORs in the two it may share with its neighbours;
//              the last block adds the 1-bit padding to a byte boundary;
//   6. stuff:  per 16 KB of stream the 0xFF count, a prefix sum over those, and
//              the copy that inserts a 0x00 after every 0xFF (staged in LDS, so
//              the stores are contiguous).
// The host reads the symbol counts once to build the tables, then the two
// totals (bits, stuffed bytes), and copies the coded bytes behind the headers.
// Scratch is sized for the largest possible stream of the frame, so no pass
// waits for the host to learn the actual size.

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
constexpr int kBlocksPerWave = 8;
constexpr int kMcuPerWave = 4;
constexpr int kGroupBlocks = kWaves * kBlocksPerWave;
// A block codes at most 27 DC bits and 63 AC symbols of at most 16 + 15 bits
// (a ZRL only replaces a nonzero coefficient): < 1985 bits.  A workgroup's
// LDS image holds 16 such blocks behind an offset of up to 31 bits, the 7 bits
// of padding and the word after the last that an OR may touch.
constexpr int kMaxBlockBits = 2048;
constexpr int kPackWords = kGroupBlocks * kMaxBlockBits / 32 + 2;
constexpr int kStuffPerThread = 16;       // bytes of stream per thread in the stuffing passes
constexpr int kStuffChunk = kThreads * kStuffPerThread;
constexpr int kHistCopies = 64;           // symbol counts kept in this many copies: fewer atomics per address
constexpr int kTopItems = 16;             // items per thread of the one-workgroup prefix sum

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

// nz: ballot of the block's nonzero lanes; prev_dc: the DC of the same
// component in the previous MCU (lane 0 only).
__device__ inline LaneSym lane_symbol(int v, int prev_dc, unsigned long long nz, int chroma, int lane) {
    LaneSym s{-1, 0, 0, 0, 0u};
    if (lane == 0) {
        const int diff = v - prev_dc;
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

// The wave's kBlocksPerWave blocks, first block b0: coefficients of this lane and
// the previous-MCU DC for lane 0, all loads issued before any is used.
struct WaveBlocks {
    int v[kBlocksPerWave];
    int prev[kBlocksPerWave];
};

__device__ inline WaveBlocks load_blocks(const int16_t* __restrict__ coef, int b0, int n_blocks, int lane) {
    WaveBlocks w;
    for (int i = 0; i < kBlocksPerWave; ++i) {
        const int b = b0 + i;
        const int16_t* blk = coef + (size_t)b * 64;
        w.v[i] = b < n_blocks ? blk[lane] : 0;
        w.prev[i] = (lane == 0 && b < n_blocks && b >= 3) ? blk[-3 * 64] : 0;
    }
    return w;
}

__device__ inline unsigned lane_bits(const LaneSym& s, const uint32_t* C) {
    if (s.table < 0) return 0;
    const uint32_t* t = C + s.table * 256;
    return (unsigned)s.zrl * (t[0xF0] >> 16) + (t[s.sym] >> 16) + (unsigned)s.size;
}

// Inclusive prefix sum over the 64 lanes by DPP: a scan inside each row of 16
// lanes (row_shr 1, 2, 4, 8; lanes whose source lies in another row add 0),
// then the last lane of row 0 (and row 2) added into row 1 (and row 3), then
// lane 31 into rows 2 and 3.
template <int CTRL, int ROWS>
__device__ inline unsigned dpp_add(unsigned v) {
    return v + (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}

__device__ inline unsigned wave_incl_scan_dpp(unsigned v) {
    v = dpp_add<0x111, 0xF>(v);
    v = dpp_add<0x112, 0xF>(v);
    v = dpp_add<0x114, 0xF>(v);
    v = dpp_add<0x118, 0xF>(v);
    v = dpp_add<0x142, 0xA>(v);            // row_bcast:15
    v = dpp_add<0x143, 0xC>(v);            // row_bcast:31
    return v;
}

__device__ inline unsigned long long wave_incl_scan64(unsigned long long v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum over the workgroup's threads; *total: the sum of all.
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

// ---- 1. coefficients ----

__global__ __launch_bounds__(kThreads) void jpeg_coef_kernel(const uint8_t* __restrict__ rgba, int width, int height,
                                                             int mcu_cols, int n_mcu,
                                                             const JpegTables* __restrict__ tab,
                                                             int16_t* __restrict__ coef) {
    __shared__ int S[kWaves][3][64];
    __shared__ int T[kWaves][3][64];
    __shared__ JpegTables TB;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = lane >> 3, c = lane & 7;
    const int m0 = (blockIdx.x * kWaves + wave) * kMcuPerWave;
    for (int i = threadIdx.x; i < (int)(sizeof(JpegTables) / 4); i += kThreads)
        reinterpret_cast<int32_t*>(&TB)[i] = reinterpret_cast<const int32_t*>(tab)[i];
    // this lane's pixel of each of the wave's MCUs, all loads in flight together
    // (an MCU beyond the frame reads the last one's pixel and is not stored)
    uint32_t px[kMcuPerWave];
    for (int i = 0; i < kMcuPerWave; ++i) {
        const int mcu = min(m0 + i, n_mcu - 1);
        const int by = mcu / mcu_cols, bx = mcu - by * mcu_cols;
        const int x = min(bx * 8 + c, width - 1), y = min(by * 8 + r, height - 1);
        px[i] = *reinterpret_cast<const uint32_t*>(rgba + ((size_t)y * width + x) * 4);
    }
    __syncthreads();
    // per lane: the row pass output (y = r, u = c) needs M[c][*], the column pass (v = r, u = c) M[r][*]
    int mu[8], mv[8];
    for (int i = 0; i < 8; ++i) mu[i] = TB.dct[c * 8 + i], mv[i] = TB.dct[r * 8 + i];
    const int q0 = TB.quant[0][lane], q1 = TB.quant[1][lane], zz = TB.zz[lane];
    const unsigned r0 = TB.qinv[0][lane], r1 = TB.qinv[1][lane];
    for (int i = 0; i < kMcuPerWave; ++i) {
        const int mcu = m0 + i;
        const bool live = mcu < n_mcu;
        if (live) {
            const int R = px[i] & 255, G = (px[i] >> 8) & 255, B = (px[i] >> 16) & 255;
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
                for (int x = 0; x < 8; ++x) acc += __mul24(mu[x], S[wave][k][r * 8 + x]);   // |M| < 2^11, |s| <= 2^7
                T[wave][k][lane] = (acc + 512) >> 10;          // two fractional bits kept
            }
        __syncthreads();
        if (live)
            for (int k = 0; k < 3; ++k) {
                int acc = 0;
                for (int y = 0; y < 8; ++y) acc += __mul24(mv[y], T[wave][k][y * 8 + c]);   // |T| < 2^12
                const int f = (acc + 8192) >> 14;
                // |f| <= 1024 for 8-bit samples, so the dividend stays below 2^12 and the
                // reciprocal product below 2^32 (24-bit operands)
                const int q = k ? q1 : q0;
                const unsigned a = (unsigned)((f < 0 ? -f : f) + (q >> 1));
                const int mag = (int)(__umul24(a, k ? r1 : r0) >> 20);
                coef[((size_t)mcu * 3 + k) * 64 + zz] = (int16_t)(f < 0 ? -mag : mag);
            }
    }
}

// ---- 2. symbol counts ----

__global__ __launch_bounds__(kThreads) void jpeg_hist_kernel(const int16_t* __restrict__ coef, int n_blocks,
                                                             uint32_t* __restrict__ hist) {
    __shared__ uint32_t H[kJpegTableCount * 256];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int b0 = (blockIdx.x * kWaves + wave) * kBlocksPerWave;
    const WaveBlocks wb = load_blocks(coef, b0, n_blocks, lane);
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads) H[i] = 0;
    __syncthreads();
    for (int i = 0; i < kBlocksPerWave; ++i) {
        const int b = b0 + i;
        const unsigned long long nz = __ballot(wb.v[i] != 0);
        if (b >= n_blocks) break;
        const LaneSym s = lane_symbol(wb.v[i], wb.prev[i], nz, (b % 3) != 0, lane);
        if (s.table >= 0) {
            atomicAdd(&H[s.table * 256 + s.sym], 1u);
            if (s.zrl) atomicAdd(&H[s.table * 256 + 0xF0], (unsigned)s.zrl);
        }
    }
    __syncthreads();
    uint32_t* copy = hist + (blockIdx.x % kHistCopies) * (kJpegTableCount * 256);
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads)
        if (H[i]) atomicAdd(&copy[i], H[i]);
}

// Sum of the copies into out, leaving the copies zero for the next frame.
__global__ __launch_bounds__(kThreads) void jpeg_hist_reduce_kernel(uint32_t* __restrict__ hist,
                                                                    uint32_t* __restrict__ out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    uint32_t v[kHistCopies];
    for (int c = 0; c < kHistCopies; ++c) v[c] = hist[c * kJpegTableCount * 256 + i];
    uint32_t sum = 0;
    for (int c = 0; c < kHistCopies; ++c) {
        sum += v[c];
        if (v[c]) hist[c * kJpegTableCount * 256 + i] = 0u;
    }
    out[i] = sum;
}

// ---- 3. bits per block and per workgroup ----

__global__ __launch_bounds__(kThreads) void jpeg_bits_kernel(const int16_t* __restrict__ coef, int n_blocks,
                                                             const uint32_t* __restrict__ lens,
                                                             uint32_t* __restrict__ bits,
                                                             unsigned long long* __restrict__ group_bits) {
    __shared__ uint32_t LN[kJpegTableCount * 256 / 4];
    __shared__ unsigned WS[kWaves];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int b0 = (blockIdx.x * kWaves + wave) * kBlocksPerWave;
    const WaveBlocks wb = load_blocks(coef, b0, n_blocks, lane);
    static_assert(kJpegTableCount * 256 / 4 == kThreads, "one word of four code lengths per thread");
    LN[threadIdx.x] = lens[threadIdx.x];
    __syncthreads();
    const uint8_t* L8 = reinterpret_cast<const uint8_t*>(LN);
    // each block's bits, then the eight wave sums side by side
    unsigned nb[kBlocksPerWave];
    for (int i = 0; i < kBlocksPerWave; ++i) {
        const int b = b0 + i;
        const unsigned long long nz = __ballot(wb.v[i] != 0);
        nb[i] = 0;
        if (b >= n_blocks) continue;
        const LaneSym s = lane_symbol(wb.v[i], wb.prev[i], nz, (b % 3) != 0, lane);
        if (s.table >= 0) {
            const uint8_t* t = L8 + s.table * 256;
            nb[i] = (unsigned)s.zrl * t[0xF0] + t[s.sym] + (unsigned)s.size;
        }
    }
    for (int i = 0; i < kBlocksPerWave; ++i)
        nb[i] = (unsigned)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(nb[i]), 63);
    unsigned wave_total = 0;
    for (int i = 0; i < kBlocksPerWave; ++i) {
        if (b0 + i >= n_blocks) break;
        if (lane == 0) bits[b0 + i] = nb[i];
        wave_total += nb[i];
    }
    if (lane == 0) WS[wave] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long g = 0;
        for (int w = 0; w < kWaves; ++w) g += WS[w];
        group_bits[blockIdx.x] = g;
    }
}

// ---- 4. one workgroup: exclusive prefix sum in place, total behind ----
// With `words`, also clears the stream word at every start offset that is not
// word aligned: the two workgroups meeting there both OR into it.

__global__ __launch_bounds__(kThreads) void scan_top_kernel(unsigned long long* __restrict__ part, long long n_parts,
                                                            unsigned long long* __restrict__ total,
                                                            uint32_t* __restrict__ words) {
    unsigned long long carry = 0;
    for (long long c0 = 0; c0 < n_parts; c0 += (long long)kThreads * kTopItems) {
        const long long i0 = c0 + (long long)threadIdx.x * kTopItems;
        unsigned long long v[kTopItems], sum = 0;
        for (int k = 0; k < kTopItems; ++k) {
            v[k] = i0 + k < n_parts ? part[i0 + k] : 0ull;
            sum += v[k];
        }
        unsigned long long all;
        unsigned long long ex = carry + block_excl_scan(sum, &all);
        for (int k = 0; k < kTopItems; ++k)
            if (i0 + k < n_parts) {
                part[i0 + k] = ex;
                if (words && (ex & 31)) words[ex >> 5] = 0u;
                ex += v[k];
            }
        carry += all;
    }
    if (threadIdx.x == 0) *total = carry;
}

// ---- 5. bit packing ----

// OR n (1..32) bits of val, most significant first, in at bit position q of W.
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

__global__ __launch_bounds__(kThreads) void jpeg_pack_kernel(const int16_t* __restrict__ coef, int n_blocks,
                                                             const uint32_t* __restrict__ codes,
                                                             const uint32_t* __restrict__ bits,
                                                             const unsigned long long* __restrict__ group_start,
                                                             uint32_t* __restrict__ words) {
    __shared__ uint32_t C[kJpegTableCount * 256];
    __shared__ uint32_t W[kPackWords];
    __shared__ unsigned BB[kGroupBlocks];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g0 = blockIdx.x * kGroupBlocks;
    const int b0 = g0 + wave * kBlocksPerWave;
    const WaveBlocks wb = load_blocks(coef, b0, n_blocks, lane);
    const unsigned long long p0 = group_start[blockIdx.x];
    const int off0 = (int)(p0 & 31);
    for (int i = threadIdx.x; i < kJpegTableCount * 256; i += kThreads) C[i] = codes[i];
    for (int i = threadIdx.x; i < kPackWords; i += kThreads) W[i] = 0u;
    if (threadIdx.x < kGroupBlocks) BB[threadIdx.x] = g0 + threadIdx.x < n_blocks ? bits[g0 + threadIdx.x] : 0u;
    __syncthreads();
    int start = off0;                       // local bit position of the wave's first block
    for (int j = 0; j < wave * kBlocksPerWave; ++j) start += (int)BB[j];
    const bool last_group = g0 + kGroupBlocks >= n_blocks;
    // the symbols of the wave's blocks, then their lane offsets by eight scans side by side
    LaneSym sy[kBlocksPerWave];
    unsigned ex[kBlocksPerWave];
    for (int i = 0; i < kBlocksPerWave; ++i) {
        const int b = b0 + i;
        const unsigned long long nz = __ballot(wb.v[i] != 0);
        sy[i] = b < n_blocks ? lane_symbol(wb.v[i], wb.prev[i], nz, (b % 3) != 0, lane) : LaneSym{-1, 0, 0, 0, 0u};
        ex[i] = lane_bits(sy[i], C);
    }
    unsigned nb[kBlocksPerWave];
    for (int i = 0; i < kBlocksPerWave; ++i) nb[i] = ex[i];
    for (int i = 0; i < kBlocksPerWave; ++i) ex[i] = wave_incl_scan_dpp(ex[i]);
    for (int i = 0; i < kBlocksPerWave; ++i) {
        const LaneSym& s = sy[i];
        int q = start + (int)(ex[i] - nb[i]);
        if (s.table >= 0) {
            const uint32_t* t = C + s.table * 256;
            const uint32_t z = t[0xF0];
            for (int k = 0; k < s.zrl; ++k) {
                lds_put(W, q, z & 0xFFFFu, (int)(z >> 16));
                q += (int)(z >> 16);
            }
            const uint32_t e = t[s.sym];
            lds_put(W, q, ((e & 0xFFFFu) << s.size) | s.extra, (int)(e >> 16) + s.size);
        }
        start += (int)BB[wave * kBlocksPerWave + i];
    }
    // the group's end, and the padding behind the frame's last block
    int end = off0;
    for (int j = 0; j < kGroupBlocks; ++j) end += (int)BB[j];
    if (last_group) {
        const int pad = (8 - (end - off0 + (int)(p0 & 7)) % 8) % 8;    // to a byte boundary of the stream
        if (pad && threadIdx.x == 0) lds_put(W, end, (1u << pad) - 1u, pad);
        end += pad;
    }
    __syncthreads();
    const int nw = (end + 31) >> 5;
    const long long base = (long long)(p0 >> 5);
    for (int w = threadIdx.x; w < nw; w += kThreads) {
        // a word is shared with the group before (unaligned start) or after (unaligned end, not the last group)
        const bool shared = (w == 0 && off0 != 0) || (w == nw - 1 && (end & 31) != 0 && !last_group);
        if (shared)
            atomicOr(&words[base + w], W[w]);
        else
            words[base + w] = W[w];
    }
}

// ---- 6. byte stuffing ----

__device__ inline uint32_t word_byte(uint32_t w, int k) { return (w >> (24 - 8 * k)) & 0xFFu; }

// The thread's 16 bytes of stream from byte k0 (16-byte aligned) and how many are 0xFF.
__device__ inline unsigned load_stream(const uint32_t* __restrict__ words, unsigned long long k0,
                                       unsigned long long n_bytes, uint32_t (&w)[4]) {
    const uint4 x = *reinterpret_cast<const uint4*>(words + (k0 >> 2));
    w[0] = x.x, w[1] = x.y, w[2] = x.z, w[3] = x.w;
    unsigned n = 0;
    for (int i = 0; i < kStuffPerThread; ++i)
        if (k0 + i < n_bytes && word_byte(w[i >> 2], i & 3) == 0xFFu) ++n;
    return n;
}

__global__ __launch_bounds__(kThreads) void stuff_count_kernel(const uint32_t* __restrict__ words,
                                                               const unsigned long long* __restrict__ total_bits,
                                                               unsigned long long* __restrict__ counts) {
    const unsigned long long n_bytes = (*total_bits + 7) / 8;
    const unsigned long long c0 = (unsigned long long)blockIdx.x * kStuffChunk;
    if (c0 >= n_bytes) {
        if (threadIdx.x == 0) counts[blockIdx.x] = 0;
        return;
    }
    const unsigned long long k0 = c0 + threadIdx.x * kStuffPerThread;
    uint32_t w[4];
    const unsigned n = k0 < n_bytes ? load_stream(words, k0, n_bytes, w) : 0u;
    unsigned long long all;
    block_excl_scan(n, &all);
    if (threadIdx.x == 0) counts[blockIdx.x] = all;
}

// Copies the workgroup's chunk of stream with a 0x00 behind every 0xFF: the
// bytes are placed in LDS first, then stored as aligned words (bytes at the ends).
__global__ __launch_bounds__(kThreads) void stuff_write_kernel(const uint32_t* __restrict__ words,
                                                               const unsigned long long* __restrict__ total_bits,
                                                               const unsigned long long* __restrict__ ff_before,
                                                               uint8_t* __restrict__ out) {
    __shared__ uint8_t L[2 * kStuffChunk];
    const unsigned long long n_bytes = (*total_bits + 7) / 8;
    const unsigned long long c0 = (unsigned long long)blockIdx.x * kStuffChunk;
    if (c0 >= n_bytes) return;
    const unsigned long long k0 = c0 + threadIdx.x * kStuffPerThread;
    uint32_t w[4];
    const unsigned n = k0 < n_bytes ? load_stream(words, k0, n_bytes, w) : 0u;
    unsigned long long all;
    unsigned pos = (unsigned)(threadIdx.x * kStuffPerThread + block_excl_scan(n, &all));
    if (k0 < n_bytes)
        for (int i = 0; i < kStuffPerThread; ++i) {
            if (k0 + i >= n_bytes) break;
            const uint32_t v = word_byte(w[i >> 2], i & 3);
            L[pos++] = (uint8_t)v;
            if (v == 0xFFu) L[pos++] = 0;
        }
    __syncthreads();
    const unsigned len = (unsigned)(std::min<unsigned long long>(kStuffChunk, n_bytes - c0) + all);
    uint8_t* dst = out + c0 + ff_before[blockIdx.x];
    const unsigned head = std::min(len, (unsigned)((4 - ((uintptr_t)dst & 3)) & 3));
    if (threadIdx.x < head) dst[threadIdx.x] = L[threadIdx.x];
    const unsigned n4 = (len - head) / 4;
    uint32_t* d4 = reinterpret_cast<uint32_t*>(dst + head);
    for (unsigned i = threadIdx.x; i < n4; i += kThreads) {
        const unsigned q = head + 4 * i;
        d4[i] = (uint32_t)L[q] | ((uint32_t)L[q + 1] << 8) | ((uint32_t)L[q + 2] << 16) | ((uint32_t)L[q + 3] << 24);
    }
    const unsigned t0 = head + 4 * n4;
    if (threadIdx.x < len - t0) dst[t0 + threadIdx.x] = L[t0 + threadIdx.x];
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

struct JpegWork {
    JpegTables* tables = nullptr;        // device
    uint32_t* codes = nullptr;           // device [4][256]
    uint32_t* hist = nullptr;            // device [kHistCopies][4][256], zero between frames
    uint32_t* hist_sum = nullptr;        // device [4][256]
    uint32_t* lens = nullptr;            // device [4][256] code lengths, bytes
    unsigned long long* totals = nullptr;  // device [2]: bit total, 0xFF total
    uint32_t* host_hist = nullptr;       // pinned [4][256]
    unsigned long long* host_totals = nullptr;  // pinned [2]
    uint32_t* host_codes = nullptr;      // pinned [4][256]
    uint8_t* host_lens = nullptr;        // pinned [4][256]
    uint8_t* host_out = nullptr;         // pinned staging of the coded bytes
    size_t host_out_cap = 0;
    JpegTables host_tables{};
    int quality = -1;
    void* buf[6] = {};
    size_t cap[6] = {};
    unsigned generation = 0;             // bumped whenever a scratch buffer moves
    // the two device segments between host round trips, replayed as graphs
    hipStream_t capture = nullptr;
    hipGraphExec_t seg_a = nullptr, seg_b = nullptr;
    const void* a_rgba = nullptr;
    int a_width = 0, a_height = 0;
    int b_blocks = 0;
    unsigned a_gen = ~0u, b_gen = ~0u;
};

namespace {

enum Buf { B_COEF = 0, B_BITS, B_GROUP, B_WORDS, B_STUFF, B_OUT };

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
    ++w->generation;
    return e;
}

// Replays *exec on stream s, first capturing `enqueue` into it on the work's
// capture stream when `fresh` is false.
template <class F>
hipError_t replay(JpegWork* w, hipGraphExec_t* exec, bool fresh, hipStream_t s, F enqueue) {
    if (!fresh || !*exec) {
        if (*exec) {
            hipGraphExecDestroy(*exec);
            *exec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(w->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        e = enqueue(w->capture);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(w->capture, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) {
            *exec = nullptr;
            return e;
        }
    }
    return hipGraphLaunch(*exec, s);
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
    if (w->hist_sum) hipFree(w->hist_sum);
    if (w->lens) hipFree(w->lens);
    if (w->host_lens) hipHostFree(w->host_lens);
    if (w->seg_a) hipGraphExecDestroy(w->seg_a);
    if (w->seg_b) hipGraphExecDestroy(w->seg_b);
    if (w->capture) hipStreamDestroy(w->capture);
    if (w->totals) hipFree(w->totals);
    if (w->host_hist) hipHostFree(w->host_hist);
    if (w->host_totals) hipHostFree(w->host_totals);
    if (w->host_codes) hipHostFree(w->host_codes);
    if (w->host_out) hipHostFree(w->host_out);
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
    const int n_mcu = mcu_cols * mcu_rows, n_blocks = 3 * n_mcu;
    // symbol counts are 32-bit (at most 64 symbols per block), workgroup bit ranges int
    if ((long long)n_blocks * 64 >= (1LL << 32))
        return fail(ISAAC_ERR_INVALID_ARGUMENT, "frame too large for one JPEG encode", hipSuccess);

    if (!w->tables) {
        JPEG_TRY(hipMalloc(&w->tables, sizeof(JpegTables)));
        JPEG_TRY(hipMalloc(&w->codes, kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipMalloc(&w->hist, kHistCopies * kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipMalloc(&w->hist_sum, kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipMalloc(&w->lens, kJpegTableCount * 256));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_lens), kJpegTableCount * 256));
        fill_u32_kernel<<<64, 256, 0, s>>>(w->hist, kHistCopies * kJpegTableCount * 256);
        JPEG_TRY(hipGetLastError());
        JPEG_TRY(hipMalloc(&w->totals, 2 * sizeof(unsigned long long)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_hist), kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_codes), kJpegTableCount * 256 * sizeof(uint32_t)));
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_totals), 2 * sizeof(unsigned long long)));
        JPEG_TRY(hipStreamCreateWithFlags(&w->capture, hipStreamNonBlocking));
    }
    if (w->quality != quality) {
        jpeg_fill_tables(quality, &w->host_tables);
        JPEG_TRY(hipMemcpyAsync(w->tables, &w->host_tables, sizeof(JpegTables), hipMemcpyHostToDevice, s));
        JPEG_TRY(hipStreamSynchronize(s));
        w->quality = quality;
    }
    // scratch for the largest stream the frame can give: kMaxBlockBits per block,
    // rounded up to whole stuffing chunks, and twice that once stuffed
    const long long groups = (n_blocks + kGroupBlocks - 1) / kGroupBlocks;
    const long long max_bytes = groups * kGroupBlocks * (kMaxBlockBits / 8);
    const long long stuff_groups = (max_bytes + kStuffChunk - 1) / kStuffChunk;
    JPEG_TRY(grow(w, B_COEF, (size_t)n_blocks * 64 * sizeof(int16_t)));
    JPEG_TRY(grow(w, B_BITS, (size_t)n_blocks * sizeof(uint32_t)));
    JPEG_TRY(grow(w, B_GROUP, (size_t)groups * sizeof(unsigned long long)));
    JPEG_TRY(grow(w, B_WORDS, (size_t)stuff_groups * kStuffChunk));
    JPEG_TRY(grow(w, B_STUFF, (size_t)stuff_groups * sizeof(unsigned long long)));
    JPEG_TRY(grow(w, B_OUT, (size_t)stuff_groups * kStuffChunk * 2));
    auto* coef = static_cast<int16_t*>(w->buf[B_COEF]);
    auto* bits = static_cast<uint32_t*>(w->buf[B_BITS]);
    auto* group = static_cast<unsigned long long*>(w->buf[B_GROUP]);
    auto* words = static_cast<uint32_t*>(w->buf[B_WORDS]);
    auto* ffcnt = static_cast<unsigned long long*>(w->buf[B_STUFF]);
    auto* dst = static_cast<uint8_t*>(w->buf[B_OUT]);

    // 1-2: coefficients and symbol counts (a graph per input frame and buffer set)
    const unsigned coef_groups = (unsigned)((n_mcu + kWaves * kMcuPerWave - 1) / (kWaves * kMcuPerWave));
    const bool same_a = w->a_rgba == rgba8 && w->a_width == width && w->a_height == height && w->a_gen == w->generation;
    JPEG_TRY(replay(w, &w->seg_a, same_a, s, [&](hipStream_t st) {
        jpeg_coef_kernel<<<coef_groups, kThreads, 0, st>>>(rgba8, width, height, mcu_cols, n_mcu, w->tables, coef);
        jpeg_hist_kernel<<<(unsigned)groups, kThreads, 0, st>>>(coef, n_blocks, w->hist);
        jpeg_hist_reduce_kernel<<<kJpegTableCount * 256 / kThreads, kThreads, 0, st>>>(w->hist, w->hist_sum);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->host_hist, w->hist_sum, kJpegTableCount * 256 * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st);
        return e;
    }));
    w->a_rgba = rgba8, w->a_width = width, w->a_height = height, w->a_gen = w->generation;
    JPEG_TRY(hipStreamSynchronize(s));

    // Huffman tables
    uint8_t bitsl[4][16], vals[4][256];
    int nvals[4];
    for (int k = 0; k < kJpegTableCount; ++k) {
        uint8_t len[256];
        jpeg_code_lengths(w->host_hist + k * 256, len);
        nvals[k] = jpeg_canonical(len, w->host_codes + k * 256, bitsl[k], vals[k]);
        memcpy(w->host_lens + k * 256, len, 256);
    }

    // 3-6: bits, offsets, packing, stuffing (a graph per buffer set)
    const bool same_b = w->b_blocks == n_blocks && w->b_gen == w->generation;
    JPEG_TRY(replay(w, &w->seg_b, same_b, s, [&](hipStream_t st) {
        hipError_t e = hipMemcpyAsync(w->codes, w->host_codes, kJpegTableCount * 256 * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(w->lens, w->host_lens, kJpegTableCount * 256, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        jpeg_bits_kernel<<<(unsigned)groups, kThreads, 0, st>>>(coef, n_blocks, w->lens, bits, group);
        scan_top_kernel<<<1, kThreads, 0, st>>>(group, groups, w->totals, words);
        jpeg_pack_kernel<<<(unsigned)groups, kThreads, 0, st>>>(coef, n_blocks, w->codes, bits, group, words);
        stuff_count_kernel<<<(unsigned)stuff_groups, kThreads, 0, st>>>(words, w->totals, ffcnt);
        scan_top_kernel<<<1, kThreads, 0, st>>>(ffcnt, stuff_groups, w->totals + 1, nullptr);
        stuff_write_kernel<<<(unsigned)stuff_groups, kThreads, 0, st>>>(words, w->totals, ffcnt, dst);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->host_totals, w->totals, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
        return e;
    }));
    w->b_blocks = n_blocks, w->b_gen = w->generation;
    JPEG_TRY(hipStreamSynchronize(s));
    const size_t coded = (size_t)((w->host_totals[0] + 7) / 8 + w->host_totals[1]);

    uint8_t hdr[kJpegHeaderMax];
    const size_t hdr_len = jpeg_headers(width, height, w->host_tables, bitsl, vals, nvals, hdr);
    const size_t need = hdr_len + coded + 2;
    *out_size = need;
    if (!out || capacity < need)
        return fail(ISAAC_ERR_INVALID_ARGUMENT, "output capacity below the stream size (written to out_size)",
                    hipSuccess);
    if (coded > w->host_out_cap) {
        if (w->host_out) JPEG_TRY(hipHostFree(w->host_out));
        w->host_out = nullptr;
        w->host_out_cap = 0;
        JPEG_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->host_out), coded));
        w->host_out_cap = coded;
    }
    JPEG_TRY(hipMemcpyAsync(w->host_out, dst, coded, hipMemcpyDeviceToHost, s));
    JPEG_TRY(hipStreamSynchronize(s));
    memcpy(out, hdr, hdr_len);
    memcpy(out + hdr_len, w->host_out, coded);
    out[hdr_len + coded] = 0xFF;
    out[hdr_len + coded + 1] = 0xD9;                            // EOI
    return 0;
#undef JPEG_TRY
}

}  // namespace isaac
