// Library-private structures shared by the host runtime (isaac_api.cpp) and
// the HIP kernels (raycast.hip).  Plain data only; everything a kernel needs
// for one job is in DevJob, built on the host and copied to device memory.
#pragma once

#include <stdint.h>

#include "isaac_mi355x.h"

namespace isaac {

constexpr int kMaxSources = 8;
constexpr int kMaxOps = 8;
constexpr int kMaxClip = 8;
constexpr int kTfEntries = 256;
// A table as stored on the device: per entry j two RGBA32F rows, T[j] and
// T[j+1] - T[j] (the last difference is 0), so a lookup is one FMA per channel.
constexpr int kTfRows = 2 * kTfEntries;
// A table as the ray-casting kernels stage it in LDS: the values T[0..255] and
// a copy of T[255] (the top entry's slope is 0); a lookup forms T[j+1] - T[j] in
// FP32, the same difference the stored rows hold, so the result is unchanged
// while a workgroup's tables take half the LDS.
constexpr int kTfLds = kTfEntries + 1;
constexpr int kMaxBatch = 256;
constexpr int kBlockThreads = 256;     // 4 waves of 64

// Functor bytecode.  ADD/MUL/POW act componentwise on the first `dim`
// components, LENGTH and SUM reduce to one component; SQRT and SQUARE are
// the host's rewrites of pow(0.5) and pow(2) with all arguments equal.
enum OpKind : int32_t {
    OP_ADD = 0,
    OP_MUL = 1,
    OP_POW = 2,
    OP_LENGTH = 3,
    OP_SUM = 4,
    OP_SQRT = 5,
    OP_SQUARE = 6,
};

struct DevOp {
    int32_t kind;
    int32_t dim;          // components the op reads
    float arg[4];
};

enum DType : int32_t { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

// Source signatures with a compile-time specialized scan-point loop (all
// sources packed, strides below 2^23 bytes); anything else runs the generic
// bytecode loop.  The arithmetic, and so the image, is the same either way.
enum Signature : int32_t {
    SIG_GENERIC = 0,
    SIG_F32x1 = 1,        // one FP32 scalar
    SIG_PIC3_F32 = 2,     // FP32 scalar, FP32 3-vector, FP32 3-vector
    SIG_PIC3_F16 = 3,     // the same in FP16
    SIG_PIC3_BF16 = 4,    // the same in BF16
    SIG_IL3 = 5,          // a three-source derived volume, x fastest (DevSource layout 0)
    SIG_IL3P = 6,         // a three-source derived volume in (y, z) pairs (DevSource layout 1)
};

struct DevSource {
    uint64_t base[4];      // per component: lowest byte address it can be read at
    uint32_t num_records[4];  // per component: bytes readable from base (buffer-resource range)
    int32_t comp_off[4];   // byte offset of component c of voxel (0,0,0) from base[c]
    int32_t packed;        // components adjacent in memory: one range (index 0), one wide load
    // 0: voxel (x, y, z) at x stride[0] + y stride[1] + z stride[2] + comp_off.
    // 1 (three-source derived volumes, read only by the SIG_IL3P loop): (y, z)
    // pairs interleaved, records of 12 bytes, voxel at (z >> 1) stride[2] +
    // (y >> 1) stride[1] + x stride[0] + ((z & 1) 2 + (y & 1)) 12 + comp_off
    // (arithmetic shifts: guard index -1 lies in pair -1), so the 2 x 2 (y, z)
    // neighbours of a voxel share its 48 bytes.
    int32_t layout;
    int32_t stride[3];     // byte strides along x, y, z (layout 1: x, y pair, z pair)
    int32_t f_dim;
    int32_t dtype;
    int32_t guard;         // >= 1: corners may reach index -1 and N; 0: clamp to the border
    int32_t n_ops;
    int32_t tf_slot;       // index into the transfer-table pool
    float weight;
    float iso;             // iso value (iso-surface jobs)
    DevOp ops[kMaxOps];
};

struct DevJob {
    // camera, FP64 (host-computed basis; per-ray setup stays FP64 on the device)
    double eye[3];
    double fwd[3];
    double right[3];
    double upp[3];
    double h;              // tan(fovy/2), or ortho_height/2
    double aspect;         // width / height
    double step;
    double clip[kMaxClip][4];
    double gbox_hi[3];     // the global box [0, gbox_hi] the step grid is anchored to
    float org[3];          // index of this volume's voxel (0,0,0) in the global box (bricks)
    float orgh[3];         // org + 1/2, exact: trilinear cell coordinates are the position minus orgh
    float half_step;       // (float)step / 2, exact
    int32_t brick;         // 1: this volume is a brick of a larger global volume
    int32_t ortho;
    int32_t width, height;
    int32_t interp;
    int32_t dims[3];
    int32_t n_src;         // active sources, compacted in index order
    int32_t n_clip;
    float ert;             // early-termination threshold
    // tile decomposition of this job's image
    int32_t wave_w;        // a wave's rays form a wave_w x (64 / lanes / wave_w) block
    int32_t waves_x;       // waves per workgroup: waves_x x (4 / waves_x)
    int32_t unroll;        // scan points whose loads are issued together (1 or 2)
    int32_t lanes;         // lanes sharing one ray (1, 2, 4, 8 or 16)
    int32_t waves_hint;    // 1: run the variant compiled for at least 4 waves per SIMD
    int32_t sig;           // Signature of the active sources
    int32_t mode;          // 0 volume compositing, 1 first iso-surface
    int32_t pool;          // 1: pooled schedule requested (single-job launches with lanes >= 2)
    int32_t tiles_x, tiles_y;
    int32_t tile_begin;    // first tile index of this job in the batch
    int32_t cull[4];       // pixels [cull[0], cull[2]] x [cull[1], cull[3]] hold every ray that can meet the box
    float* out;            // device RGBA32F image
    int32_t* out_samples;  // device per-pixel sample counts or null
    float* out_depth;      // device per-pixel ray parameter of the first scan point (+inf: none) or null
    void* rays;            // device ray records over the screen rectangle (set up by a separate pass) or null
    int32_t src_index[kMaxSources];  // volume source index of each active source (host bookkeeping)
    DevSource src[kMaxSources];
};

// Launch entry points implemented in raycast.hip.
struct LaunchArgs {
    const DevJob* jobs;        // device
    int n_jobs;
    int total_tiles;
    const float* tf_pool;      // device, [slot][256][4]
    int* cursor;               // device work counter (persistent mode)
    int persistent;            // 0: one workgroup per tile; 1: grid-stride over a tile queue
    int grid;                  // workgroups launched in persistent mode
    int max_src;               // widest job's active source count (sizes the LDS tables)
    int unroll;                // scan points whose loads are issued together (kernel variant)
    int lanes;                 // lanes per ray (kernel variant); 1 when unroll > 1
    int waves_hint;            // 1: the variant compiled for at least 4 waves per SIMD
    int sig;                   // the jobs' common Signature, or -1 when they differ
    int mode;                  // 1: iso-surface jobs (all jobs of a launch share the mode)
    unsigned fill_blocks;      // blocks per job of the fill of pixels outside the screen rectangles
    int dense_setup;           // 1: set up every ray of the jobs' rectangles into DevJob::rays first
};

int launch_prepass(const LaunchArgs& a, void* stream);               // fill outside the rectangles, ray setup
// The same for one job passed by value, which the kernel also stores at dst
// (the device job block the ray-casting launch reads).
int launch_prepass_one(const DevJob& job, DevJob* dst, unsigned fill_blocks, int dense, void* stream);
int launch_raycast(const LaunchArgs& a, void* stream);               // returns hipError_t
int launch_reset_counter(int* counter, void* stream);
// Pooled schedule of one job (lanes >= 2): ray setup with compaction into
// `rays` (ray_record_bytes() per pixel), then a resident kernel handing the
// compacted rays to lane groups.  counters: 2 device ints.
int launch_raycast_pooled(const DevJob* job_dev, int width, int height, const float* tf_pool, int max_src, int sig,
                          int lanes, int hint, void* rays, int* counters, int n_cu, void* stream);
size_t ray_record_bytes();
int launch_strided_copy(const void* const* src_comp, const int64_t* src_stride, void* dst,
                        const int64_t* dst_stride, int esize, int f_dim, const int32_t lo[3],
                        const int32_t ext[3], void* stream);
int raycast_occupancy(int* blocks_per_cu);
// Device scratch of the render calls that allocate nothing (ray records of the
// set-up pass): a static array of kNoAllocScratchBytes per device.  Looks up the
// current device's copy (call with `device` current) once per device; *ptr is
// its device address.
constexpr size_t kNoAllocScratchBytes = ISAAC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
int noalloc_scratch(int device, void** ptr);

// Derived volume: the functor-chain output of up to 4 sources at every voxel
// of [-g, N-1+g]^3, interleaved (n floats per voxel).  paired = 0: x fastest,
// then y, then z.  paired = 1 (DevSource layout 1): rows of x records for each
// pair of (y, z) pairs, the 4 records of a (y, z) quad adjacent; stored y and
// z indices are index + gp (gp = g rounded up to even, so a stored pair holds
// an even index and the next one), ny2 x nz2 pairs.
constexpr int kMaxDerived = 4;
constexpr int kMaxKeepSets = 4;
struct DeriveArgs {
    DevSource src[kMaxDerived];   // as the ray loop would read them
    int n;                        // sources (components per voxel)
    int g;                        // guard layers covered
    int ext[3];                   // N + 2g per axis
    int paired;                   // 1: (y, z)-paired layout
    int gp;                       // g rounded up to even (paired)
    int ny2, nz2;                 // stored y and z pairs (paired)
    float org[3];                 // index of voxel (0,0,0) in the clip planes' space
    // Voxels no kept scan point can read are skipped: a voxel is derived if,
    // for at least one set, it lies within 3 voxels of every plane's kept side
    // (normalized planes; n_sets = 0: derive every voxel).
    int n_sets;
    int n_planes[kMaxKeepSets];
    float planes[kMaxKeepSets][kMaxClip][4];
    float* dst;
};
// sig: the Signature of src[0..n) (their compile-time kinds), or SIG_GENERIC
int launch_derive(const DeriveArgs& a, int sig, void* stream);
constexpr int kMaxLayers = 16;
int launch_composite(const float* const* rgba, const float* const* depth, int n_layers, int64_t n_pixels,
                     float* out, void* stream);
int launch_encode_rgba8(const float* rgba, int64_t n_pixels, const float* bg, unsigned char* out, void* stream);

}  // namespace isaac
