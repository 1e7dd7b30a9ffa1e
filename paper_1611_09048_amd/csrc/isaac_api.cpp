// Host runtime of the ray caster: the C ABI declared in include/isaac_mi355x.h.
//
// Responsibilities: validating descriptors (all-or-nothing), compiling
// functor chains to bytecode, baking transfer tables, building per-job
// parameter blocks (camera basis in FP64, clip planes, active sources),
// staging them through pinned memory, launching the kernels of raycast.hip,
// batching jobs into persistent launches replayed as hipGraphs, and the
// library-owned output images of the serving calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <string>
#include <vector>

#include "../../include/isaac_mi355x.h"
#include "host_logic.h"
#include "isaac_internal.h"
#include "jpeg_internal.h"

using namespace isaac;
using isaac::host::bake_tf;
using isaac::host::camera_basis;
using isaac::host::CameraBasis;
using isaac::host::compile_chain;
using isaac::host::CompiledChain;
using isaac::host::set_cull_rect;

namespace {

constexpr int kRingSlots = 16;
constexpr int kTfSlots = 4096;      // transfer tables resident at once (16 MiB)

struct Status {
    isaac_status code = ISAAC_OK;
    std::string msg;
};

int esize_of(int dtype) { return dtype == ISAAC_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// context state
// ---------------------------------------------------------------------------
struct SourceHost {
    isaac_source_desc desc{};
    std::string name, chain_text;
    CompiledChain chain;
    int reach = 0;                  // guard layers the kernel may read (0 or 1)
    // readable ranges of the user's memory
    uint64_t base[4] = {0, 0, 0, 0};
    uint32_t num_records[4] = {0, 0, 0, 0};
    int32_t comp_off[4] = {0, 0, 0, 0};
    int32_t stride[3] = {0, 0, 0};
    int packed = 0;
    // shadow copy for non-persistent sources
    void* shadow = nullptr;
    size_t shadow_bytes = 0;
};

struct Volume {
    bool defined = false;
    int32_t dims[3] = {0, 0, 0};
    std::vector<SourceHost> src;
    std::vector<int32_t> tf;        // current table handle per source
    // derived volume (chain outputs per voxel), rebuilt by each render call that uses it
    void* derived = nullptr;
    size_t derived_bytes = 0;
    // frozen (isaac_freeze_volume): the derived volume holds every source's
    // values and stays valid until the sources are redefined; frozen_src[s] is
    // how source s is read from it
    bool frozen = false;
    DevSource frozen_src[kMaxSources];
};

struct TfSlot {
    bool live = false;              // allocated (referenced by a handle)
    bool released = false;
    uint64_t last_use = 0;          // render sequence number that last read it
};

struct RingSlot {
    DevJob* host = nullptr;         // pinned
    DevJob* dev = nullptr;
    int* cursor = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    // graph cache
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int g_jobs = -1, g_tiles = -1, g_grid = -1, g_src = -1, g_unroll = -1, g_lanes = -1, g_hint = -1, g_sig = -3;
    unsigned g_fill = 0;
    int g_dense = -1;
};

struct Pending {
    uint64_t seq;
    hipEvent_t ev;
    bool pooled = true;             // false: a staging-ring event, not returned to the event pool
};

struct Ticket {
    uint64_t id;
    float* out = nullptr;
    size_t bytes = 0;
    int width = 0, height = 0;
    hipEvent_t ev = nullptr;
    bool done = false;
};

// Serving images: one device allocation of the memory budget, made at the
// first submission and carved into images first fit (256-byte granules, free
// neighbours merged on release), so no request allocates or frees device
// memory (hipFree would wait for the whole device).
class ImageArena {
public:
    static constexpr size_t kGranule = 256;
    bool ready() const { return base_ != nullptr; }
    bool init(size_t bytes) {
        bytes = bytes / kGranule * kGranule;
        if (bytes == 0 || hipMalloc((void**)&base_, bytes) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        size_ = bytes;
        free_.clear();
        free_[0] = bytes;
        return true;
    }
    void destroy() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        size_ = 0;
        free_.clear();
    }
    static size_t rounded(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }
    // first free run that fits; nullptr if none does
    float* take(size_t bytes) {
        bytes = rounded(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, left = it->second - bytes;
            free_.erase(it);
            if (left) free_[off + bytes] = left;
            return reinterpret_cast<float*>(base_ + off);
        }
        return nullptr;
    }
    void give(float* p, size_t bytes) {
        bytes = rounded(bytes);
        size_t off = (size_t)(reinterpret_cast<char*>(p) - base_);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
};

struct TileShape {
    int wave_w = 8, waves_x = 2, unroll = 1, lanes = 1, waves_hint = 0, pool = 0;
};

}  // namespace

struct isaac_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> serve_streams;
    int serve_rr = 0;
    int n_cu = 0;
    int blocks_per_cu = 1;
    size_t budget = 0, used = 0;
    int max_inflight = 64;
    std::vector<Volume> volumes;
    // transfer-table pool
    float* tf_pool = nullptr;
    int tf_capacity = 0;
    std::vector<TfSlot> tf_slots;
    // job staging ring
    RingSlot ring[kRingSlots];
    int ring_next = 0;
    // completion tracking
    uint64_t seq = 0, completed = 0;
    std::deque<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    // timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
    // serving
    std::map<uint64_t, Ticket> tickets;
    ImageArena images;                 // served images, within the memory budget
    uint64_t next_ticket = 1;
    void* enc_buf = nullptr;           // RGBA8 staging of isaac_read_image_rgba8 / _jpeg
    isaac::JpegWork* jpeg = nullptr;   // JPEG encoder scratch, created on first use
    size_t enc_bytes = 0;
    void* pool_rays = nullptr;         // compacted rays of the pooled schedule
    size_t pool_bytes = 0;
    int* pool_counters = nullptr;      // [appended rays, handed-out rays]
    void* noalloc_scratch = nullptr;   // this device's static scratch (ray records of isaac_render_noalloc)
    TileShape shapes[16];
    std::string last_error;
    bool sticky = false;
};

namespace {

thread_local std::string g_init_error;

isaac_status set_err(isaac_context* ctx, isaac_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) {
        ctx->last_error = buf;
        if (code == ISAAC_ERR_DEVICE) ctx->sticky = true;
    }
    return code;
}

// Device pointers are read and written a whole element at a time: RGBA32F
// pixels 16 bytes, counts, depths and RGBA8 pixels 4 bytes.
inline bool aligned_to(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

#define HIP_TRY(ctx, expr)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return set_err(ctx, ISAAC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

hipEvent_t get_event(isaac_context* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void put_event(isaac_context* ctx, hipEvent_t e) {
    if (e) ctx->event_pool.push_back(e);
}

bool is_current(const isaac_context* ctx, int32_t slot);

// Retire finished renders; reclaim released tables no queued render reads.
void update_completed(isaac_context* ctx) {
    while (!ctx->pending.empty()) {
        Pending& p = ctx->pending.front();
        if (hipEventQuery(p.ev) != hipSuccess) break;
        ctx->completed = p.seq;
        if (p.pooled) put_event(ctx, p.ev);
        ctx->pending.pop_front();
    }
    for (size_t i = 0; i < ctx->tf_slots.size(); ++i) {
        TfSlot& s = ctx->tf_slots[i];
        if (s.live && s.released && s.last_use <= ctx->completed && !is_current(ctx, (int32_t)i)) s = TfSlot();
    }
}

isaac_status check_ctx(isaac_context* ctx) {
    if (!ctx) return ISAAC_ERR_INVALID_ARGUMENT;
    if (ctx->sticky) return ISAAC_ERR_DEVICE;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    return ISAAC_OK;
}

bool is_current(const isaac_context* ctx, int32_t slot) {
    for (const Volume& v : ctx->volumes)
        for (int32_t t : v.tf)
            if (t == slot) return true;
    return false;
}

// Allocate a slot and upload a table.  Slot 0 is the all-zero table.  A
// reclaimed slot is no longer read by any queued render, so the synchronous
// upload cannot race with a kernel.
isaac_status new_tf_slot(isaac_context* ctx, const float* table, int32_t* handle) {
    update_completed(ctx);
    int slot = -1;
    for (int i = 1; i < ctx->tf_capacity; ++i)
        if (!ctx->tf_slots[i].live) {
            slot = i;
            break;
        }
    if (slot < 0)
        return set_err(ctx, ISAAC_ERR_OUT_OF_MEMORY, "all %d transfer tables are live; release some", ctx->tf_capacity);
    // device layout: per entry the value and the difference to the next entry (FP32, as the lookup uses it;
    // the last entry's difference is 0, and the lookup reads it at the top of the range)
    float rows[kTfRows * 4];
    for (int j = 0; j < kTfEntries; ++j)
        for (int c = 0; c < 4; ++c) {
            rows[8 * j + c] = table[4 * j + c];
            rows[8 * j + 4 + c] = j + 1 < kTfEntries ? table[4 * (j + 1) + c] - table[4 * j + c] : 0.0f;
        }
    HIP_TRY(ctx, hipMemcpy(ctx->tf_pool + (size_t)slot * kTfRows * 4, rows, kTfRows * 4 * sizeof(float),
                           hipMemcpyHostToDevice));
    ctx->tf_slots[slot] = TfSlot();
    ctx->tf_slots[slot].live = true;
    *handle = slot;
    return ISAAC_OK;
}

// Byte ranges the kernel may read for one source: one range per component,
// or a single range when the components are interleaved (packed).
isaac_status derive_layout(isaac_context* ctx, const int32_t dims[3], SourceHost& s) {
    const isaac_source_desc& d = s.desc;
    const int es = esize_of(d.dtype);
    s.reach = d.guard >= 1 ? 1 : 0;
    int64_t mn = 0, mx = 0;   // reachable voxel offsets relative to voxel (0,0,0)
    for (int a = 0; a < 3; ++a) {
        const int64_t e0 = -(int64_t)s.reach * d.stride[a];
        const int64_t e1 = (int64_t)(dims[a] - 1 + s.reach) * d.stride[a];
        mn += std::min(e0, e1);
        mx += std::max(e0, e1);
        const int64_t ext = (int64_t)(dims[a] + 2 * s.reach) * std::llabs(d.stride[a]);
        if (ext >= ((int64_t)1 << 31))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': axis %d spans 2 GiB or more", s.name.c_str(), a);
        s.stride[a] = (int32_t)d.stride[a];
    }
    const char* c0 = static_cast<const char*>(d.comp[0]);
    s.packed = 1;
    for (int c = 1; c < d.f_dim; ++c)
        if (static_cast<const char*>(d.comp[c]) - c0 != (int64_t)c * es) s.packed = 0;
    const int64_t span = mx - mn + (s.packed ? (int64_t)d.f_dim * es : es);
    if (span <= 0 || span >= ((int64_t)1 << 31))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': readable extent %lld bytes must be below 2 GiB",
                       s.name.c_str(), (long long)span);
    for (int c = 0; c < 4; ++c) {
        s.base[c] = 0;
        s.num_records[c] = 0;
        s.comp_off[c] = 0;
    }
    if (s.packed) {
        s.base[0] = (uint64_t)(reinterpret_cast<uintptr_t>(c0) + mn);
        s.num_records[0] = (uint32_t)span;
        for (int c = 0; c < d.f_dim; ++c) s.comp_off[c] = (int32_t)(-mn + (int64_t)c * es);
    } else {
        for (int c = 0; c < d.f_dim; ++c) {
            s.base[c] = (uint64_t)(reinterpret_cast<uintptr_t>(d.comp[c]) + mn);
            s.num_records[c] = (uint32_t)span;
            s.comp_off[c] = (int32_t)(-mn);
        }
    }
    return ISAAC_OK;
}

bool finite3(const double v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Which compile-time specialized loop (if any) fits the job's active sources.
int32_t signature_of(const DevJob& dj) {
    if (dj.n_src == 3) {
        // the three sources of one derived volume (either layout), in order
        const DevSource* d = dj.src;
        bool il = true;
        for (int s = 0; s < 3; ++s)
            il = il && d[s].f_dim == 1 && d[s].dtype == DT_F32 && d[s].n_ops == 0 && d[s].base[0] == d[0].base[0] &&
                 d[s].num_records[0] == d[0].num_records[0] && d[s].comp_off[0] == d[0].comp_off[0] + 4 * s &&
                 d[s].guard >= 1 && d[s].layout == d[0].layout && d[s].stride[0] == (d[s].layout ? 48 : 12) &&
                 d[s].stride[1] == d[0].stride[1] && d[s].stride[2] == d[0].stride[2] && d[s].stride[1] < (1 << 23) &&
                 d[s].stride[2] < (1 << 23);
        if (il) return d[0].layout ? SIG_IL3P : SIG_IL3;
    }
    int kinds[kMaxSources];
    for (int s = 0; s < dj.n_src; ++s) {
        const DevSource& d = dj.src[s];
        bool small = true;
        for (int a = 0; a < 3; ++a) small = small && std::abs((int64_t)d.stride[a]) < (1 << 23);
        if (!d.packed || !small || (d.f_dim != 1 && d.f_dim != 3)) return SIG_GENERIC;
        if (dj.n_src == 3 && d.guard < 1) return SIG_GENERIC;   // the three-source loops assume guard layers
        kinds[s] = d.dtype * 2 + (d.f_dim == 3 ? 1 : 0);   // dtype-major: F32x1=0, F32x3=1, F16x1=2, ...
    }
    if (dj.n_src == 1 && kinds[0] == 0) return SIG_F32x1;
    if (dj.n_src == 3 && kinds[1] == kinds[0] + 1 && kinds[2] == kinds[1] && kinds[0] % 2 == 0) {
        if (kinds[0] == 0) return SIG_PIC3_F32;
        if (kinds[0] == 2) return SIG_PIC3_F16;
        if (kinds[0] == 4) return SIG_PIC3_BF16;
    }
    return SIG_GENERIC;
}

// Tile decomposition of a job for a launch running `lanes` lanes per ray.
// Tiles cover only the job's screen rectangle (cull); the pixels outside it
// are cleared by a fill kernel.
void set_tiles(DevJob& dj, int lanes, int unroll) {
    dj.lanes = lanes;
    dj.unroll = lanes > 1 ? 1 : unroll;
    const int rays = 64 / lanes;
    if (dj.wave_w > rays) dj.wave_w = rays;
    const int tw = dj.wave_w * dj.waves_x, th = (rays / dj.wave_w) * (4 / dj.waves_x);
    const int rw = std::max(0, dj.cull[2] - dj.cull[0] + 1), rh = std::max(0, dj.cull[3] - dj.cull[1] + 1);
    dj.tiles_x = (rw + tw - 1) / tw;
    dj.tiles_y = rw > 0 ? (rh + th - 1) / th : 0;
}

int size_class_of(int w, int h) {
    int m = std::max(w, h), c = 0;
    while ((1 << c) < m && c < 15) ++c;
    return c;
}

// Validate one job and build its device block (without writing anything shared).
isaac_status build_job(isaac_context* ctx, const isaac_render_desc& j, bool need_out, DevJob& dj,
                       int* n_active_out) {
    if (j.volume_id < 0 || j.volume_id >= (int)ctx->volumes.size() || !ctx->volumes[j.volume_id].defined)
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "volume %d is not defined", j.volume_id);
    const Volume& v = ctx->volumes[j.volume_id];
    if (j.width < 1 || j.height < 1 || j.width > 32768 || j.height > 32768)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "image size %dx%d outside 1..32768", j.width, j.height);
    if (j.projection != ISAAC_PERSPECTIVE && j.projection != ISAAC_ORTHOGRAPHIC)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "unknown projection %d", j.projection);
    if (!finite3(j.eye) || !finite3(j.center) || !finite3(j.up))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "camera vectors must be finite");
    if (j.projection == ISAAC_PERSPECTIVE && !(j.fovy_deg > 0.0 && j.fovy_deg < 180.0))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "fovy_deg must lie in (0,180)");
    if (j.projection == ISAAC_ORTHOGRAPHIC && !(j.ortho_height > 0.0 && std::isfinite(j.ortho_height)))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "ortho_height must be positive");
    if (!(j.step > 0.0 && std::isfinite(j.step)))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "step must be positive");
    {
        const double diag = std::sqrt((double)v.dims[0] * v.dims[0] + (double)v.dims[1] * v.dims[1] +
                                      (double)v.dims[2] * v.dims[2]);
        if (diag / j.step > 1e9)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "step too small: more than 1e9 samples per ray");
    }
    if (j.interpolation != ISAAC_NEAREST && j.interpolation != ISAAC_TRILINEAR)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "unknown interpolation %d", j.interpolation);
    if (j.n_clip < 0 || j.n_clip > kMaxClip || (j.n_clip > 0 && !j.clip))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "n_clip must be 0..%d with a plane array", kMaxClip);
    if (!(j.ert_threshold >= 0.0f) || !std::isfinite(j.ert_threshold))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "ert_threshold must be >= 0");
    if (need_out && !j.out_rgba) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "out_rgba is NULL");
    if (need_out && (!aligned_to(j.out_rgba, 16) || !aligned_to(j.out_samples, 4)))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "out_rgba must be 16-byte and out_samples 4-byte aligned");
    if (!aligned_to(j.out_depth, 4)) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "out_depth must be 4-byte aligned");
    if (j.mode != ISAAC_VOLUME && j.mode != ISAAC_ISO)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "unknown render mode %d", j.mode);
    if (j.mode == ISAAC_ISO && j.brick_origin)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "iso-surface mode does not render bricks");
    if (j.mode == ISAAC_ISO && j.iso_values)
        for (int s = 0; s < (int)v.src.size(); ++s)
            if (std::isinf(j.iso_values[s]))
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "iso value of source %d is infinite", s);
    CameraBasis cb;
    std::string err;
    if (!camera_basis(j, cb, err)) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "%s", err.c_str());
    std::memset(&dj, 0, sizeof dj);
    for (int a = 0; a < 3; ++a) {
        dj.eye[a] = j.eye[a];
        dj.fwd[a] = cb.fwd[a];
        dj.right[a] = cb.right[a];
        dj.upp[a] = cb.upp[a];
        dj.dims[a] = v.dims[a];
    }
    dj.h = cb.h;
    dj.aspect = cb.aspect;
    dj.step = j.step;
    dj.half_step = 0.5f * (float)dj.step;
    dj.ortho = j.projection == ISAAC_ORTHOGRAPHIC;
    dj.width = j.width;
    dj.height = j.height;
    dj.interp = j.interpolation;
    dj.n_clip = j.n_clip;
    for (int c = 0; c < j.n_clip; ++c) {
        const isaac_clip_plane& p = j.clip[c];
        const double nn = p.n[0] * p.n[0] + p.n[1] * p.n[1] + p.n[2] * p.n[2];
        if (!(nn > 0.0) || !std::isfinite(nn) || !std::isfinite(p.d))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "clip plane %d needs a finite non-zero normal", c);
        dj.clip[c][0] = p.n[0];
        dj.clip[c][1] = p.n[1];
        dj.clip[c][2] = p.n[2];
        dj.clip[c][3] = p.d;
    }
    dj.ert = j.ert_threshold == 0.0f ? 0.999f : j.ert_threshold;
    if (j.brick_origin) {
        if (!j.global_dims) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "brick_origin needs global_dims");
        for (int a = 0; a < 3; ++a) {
            if (j.brick_origin[a] < 0 || j.global_dims[a] < 1 || j.brick_origin[a] + v.dims[a] > j.global_dims[a] ||
                j.global_dims[a] > (1 << 22))
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "brick axis %d lies outside the global box", a);
            dj.org[a] = (float)j.brick_origin[a];
            dj.orgh[a] = (float)j.brick_origin[a] + 0.5f;
            dj.gbox_hi[a] = (double)j.global_dims[a];
        }
        dj.brick = 1;
    } else {
        for (int a = 0; a < 3; ++a) {
            dj.org[a] = 0.0f;
            dj.orgh[a] = 0.5f;
            dj.gbox_hi[a] = (double)v.dims[a];
        }
        dj.brick = 0;
    }
    dj.out_depth = j.out_depth;
    set_cull_rect(dj);
    const TileShape& ts = ctx->shapes[size_class_of(j.width, j.height)];
    dj.wave_w = ts.wave_w;
    dj.waves_x = ts.waves_x;
    dj.unroll = ts.unroll;
    dj.lanes = ts.lanes;
    dj.waves_hint = ts.waves_hint;
    dj.pool = ts.pool;
    set_tiles(dj, ts.lanes, ts.unroll);
    dj.out = j.out_rgba;
    dj.out_samples = j.out_samples;
    int n_act = 0;
    for (int s = 0; s < (int)v.src.size(); ++s) {
        const SourceHost& sh = v.src[s];
        const bool en = j.enabled ? j.enabled[s] != 0 : sh.desc.enabled != 0;
        const float w = j.weights ? j.weights[s] : sh.desc.weight;
        if (!(w >= 0.0f && w <= 1.0f))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "weight of source %d must lie in [0,1]", s);
        int32_t tf = j.tf_handles ? j.tf_handles[s] : v.tf[s];
        if (tf < 0 || tf >= ctx->tf_capacity || !ctx->tf_slots[tf].live || (j.tf_handles && tf == 0))
            return set_err(ctx, ISAAC_ERR_NOT_FOUND, "transfer table handle %d of source %d is not live", tf, s);
        const float iso = j.mode == ISAAC_ISO && j.iso_values ? j.iso_values[s] : NAN;
        if (j.mode == ISAAC_ISO) {
            if (!en || std::isnan(iso)) continue;   // draws no surface: never read
        } else if (!en || w == 0.0f) {
            continue;                                // never read: a zero weight contributes exactly nothing
        }
        if (!sh.desc.comp[0] && !sh.shadow)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source %d is enabled but has no data", s);
        dj.src_index[n_act] = s;
        DevSource& ds = dj.src[n_act++];
        ds.packed = sh.packed;
        for (int c = 0; c < 4; ++c) {
            ds.base[c] = sh.base[c];
            ds.num_records[c] = sh.num_records[c];
            ds.comp_off[c] = sh.comp_off[c];
        }
        for (int a = 0; a < 3; ++a) ds.stride[a] = sh.stride[a];
        ds.f_dim = sh.desc.f_dim;
        ds.dtype = sh.desc.dtype;
        ds.guard = sh.reach;
        ds.n_ops = sh.chain.n_ops;
        for (int o = 0; o < sh.chain.n_ops; ++o) ds.ops[o] = sh.chain.ops[o];
        ds.tf_slot = tf;
        ds.weight = w;
        ds.iso = j.mode == ISAAC_ISO ? iso : 0.0f;
    }
    dj.n_src = n_act;
    dj.mode = j.mode;
    dj.sig = signature_of(dj);
    if (dj.mode == ISAAC_ISO) {
        // iso jobs run their own kernel with the runtime source loop: 8 lanes per
        // ray when the size class asks for several, else one
        dj.sig = SIG_GENERIC;
        dj.waves_hint = 0;
        dj.pool = 0;
        set_tiles(dj, ts.lanes >= 8 ? 8 : 1, 1);
    }
    *n_active_out = n_act;
    return ISAAC_OK;
}

// update() callbacks and copies of non-persistent sources for the volumes of a call
isaac_status prepare_sources(isaac_context* ctx, const isaac_render_desc* jobs, int n) {
    std::vector<int> vols;
    for (int i = 0; i < n; ++i)
        if (std::find(vols.begin(), vols.end(), jobs[i].volume_id) == vols.end()) vols.push_back(jobs[i].volume_id);
    for (int vid : vols) {
        Volume& v = ctx->volumes[vid];
        for (int s = 0; s < (int)v.src.size(); ++s) {
            SourceHost& sh = v.src[s];
            bool en = false;
            for (int i = 0; i < n; ++i)
                if (jobs[i].volume_id == vid) en = en || (jobs[i].enabled ? jobs[i].enabled[s] != 0 : sh.desc.enabled != 0);
            void* ptr = nullptr;
            for (int i = 0; i < n; ++i)
                if (jobs[i].volume_id == vid) {
                    ptr = jobs[i].update_pointer;
                    break;
                }
            if (sh.desc.update) sh.desc.update(sh.desc.user, en ? 1 : 0, ptr);
            if (!sh.desc.persistent && en) {
                const int es = esize_of(sh.desc.dtype);
                const int64_t ex = v.dims[0] + 2 * sh.reach, ey = v.dims[1] + 2 * sh.reach;
                int64_t dst_stride[3] = {(int64_t)sh.desc.f_dim * es, (int64_t)sh.desc.f_dim * es * ex,
                                         (int64_t)sh.desc.f_dim * es * ex * ey};
                char* dst0 = static_cast<char*>(sh.shadow) +
                             sh.reach * (dst_stride[0] + dst_stride[1] + dst_stride[2]);
                int32_t lo[3] = {-sh.reach, -sh.reach, -sh.reach};
                int32_t ext[3] = {v.dims[0] + 2 * sh.reach, v.dims[1] + 2 * sh.reach, v.dims[2] + 2 * sh.reach};
                int rc = launch_strided_copy(sh.desc.comp, sh.desc.stride, dst0, dst_stride, es, sh.desc.f_dim, lo, ext,
                                             ctx->stream);
                if (rc != hipSuccess)
                    return set_err(ctx, ISAAC_ERR_DEVICE, "strided copy: %s", hipGetErrorString((hipError_t)rc));
                // the next update() may reuse the buffer this copy reads
                HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            }
        }
    }
    return ISAAC_OK;
}

isaac_status acquire_slot(isaac_context* ctx, RingSlot** out) {
    RingSlot& r = ctx->ring[ctx->ring_next];
    ctx->ring_next = (ctx->ring_next + 1) % kRingSlots;
    if (r.busy) {
        HIP_TRY(ctx, hipEventSynchronize(r.done));
        r.busy = false;
    }
    *out = &r;
    return ISAAC_OK;
}

// Ray buffer and counters of the pooled schedule, grown to `bytes`.
bool ensure_pool(isaac_context* ctx, size_t bytes, hipStream_t stream) {
    if (!ctx->pool_counters && hipMalloc(&ctx->pool_counters, 2 * sizeof(int)) != hipSuccess) {
        ctx->pool_counters = nullptr;
        return false;
    }
    if (bytes <= ctx->pool_bytes) return true;
    if (ctx->pool_rays) {
        if (hipStreamSynchronize(stream) != hipSuccess) return false;
        hipFree(ctx->pool_rays);
    }
    ctx->pool_rays = nullptr;
    ctx->pool_bytes = 0;
    if (hipMalloc(&ctx->pool_rays, bytes) != hipSuccess) {
        ctx->pool_rays = nullptr;
        return false;
    }
    ctx->pool_bytes = bytes;
    return true;
}

// noalloc: the call may not allocate: the set-up pass writes its ray records
// into the context device's static scratch (the caller checked they fit), no
// pooled schedule, no hipGraph, and the staging ring's event marks completion.
isaac_status enqueue_jobs(isaac_context* ctx, const isaac_render_desc* jobs, const std::vector<DevJob>& djs,
                          int max_src, unsigned flags, hipStream_t stream, bool allow_pool, bool noalloc = false) {
    const int n = (int)djs.size();
    RingSlot* r = nullptr;
    isaac_status st = acquire_slot(ctx, &r);
    if (st) return st;
    // one kernel variant per launch: the most lanes per ray any job asks for,
    // else the deepest unroll; every job's tiles follow the launch's variant
    int lanes = 1, unroll = 1, hint = 0;
    for (const DevJob& dj : djs) lanes = std::max(lanes, (int)dj.lanes);
    for (const DevJob& dj : djs) hint = std::max(hint, (int)dj.waves_hint);
    if (lanes == 1)
        for (const DevJob& dj : djs) unroll = std::max(unroll, (int)dj.unroll);
    int tiles = 0;
    for (int i = 0; i < n; ++i) {
        r->host[i] = djs[i];
        set_tiles(r->host[i], lanes, unroll);
        r->host[i].tile_begin = tiles;
        tiles += r->host[i].tiles_x * r->host[i].tiles_y;
    }
    const uint64_t seq = ++ctx->seq;
    // mark every table read by this call
    for (const DevJob& dj : djs)
        for (int s = 0; s < dj.n_src; ++s) ctx->tf_slots[dj.src[s].tf_slot].last_use = seq;
    (void)jobs;
    LaunchArgs la;
    la.jobs = r->dev;
    la.n_jobs = n;
    la.total_tiles = tiles;
    la.tf_pool = ctx->tf_pool;
    la.cursor = r->cursor;
    la.persistent = n > 1 ? 1 : 0;
    la.grid = std::max(1, ctx->n_cu * ctx->blocks_per_cu);
    la.max_src = std::max(1, max_src);
    la.unroll = unroll;
    la.lanes = lanes;
    la.waves_hint = (lanes == 2 || lanes >= 32 || unroll > 1) ? 0 : hint;
    la.sig = djs[0].sig;
    for (const DevJob& dj : djs)
        if (dj.sig != la.sig) la.sig = -1;
    if (la.sig == SIG_GENERIC) la.sig = -1;
    la.mode = djs[0].mode;
    if (la.mode == ISAAC_ISO) {
        // the plain-source iso kernel when every source is a packed FP32 scalar without
        // functors, with guard layers and affine strides (derived volumes in x-fastest
        // order, plain scalars)
        bool plain = true;
        for (const DevJob& dj : djs)
            for (int k = 0; k < dj.n_src; ++k) {
                const DevSource& d = dj.src[k];
                plain = plain && d.packed && d.dtype == DT_F32 && d.f_dim == 1 && d.n_ops == 0 && d.guard >= 1 &&
                        d.layout == 0;
            }
        la.sig = plain ? -3 : -2;
    }
    {
        size_t maxpix = 1;
        for (const DevJob& dj : djs) maxpix = std::max(maxpix, (size_t)dj.width * dj.height);
        la.fill_blocks = (unsigned)std::min<size_t>((maxpix + 1023) / 1024, 1024);
    }
    // render calls on the context stream set up the rays in a pass of their own
    // (one lane per ray) into the context's ray buffer
    la.dense_setup = 0;
    if (noalloc) {
        size_t off = 0;
        for (int i = 0; i < n; ++i) {
            DevJob& dj = r->host[i];
            dj.rays = static_cast<char*>(ctx->noalloc_scratch) + off * ray_record_bytes();
            off += (size_t)std::max(0, dj.cull[2] - dj.cull[0] + 1) * std::max(0, dj.cull[3] - dj.cull[1] + 1);
        }
        if (off * ray_record_bytes() > kNoAllocScratchBytes)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "ray records exceed the scratch");   // checked before
        la.dense_setup = off > 0 ? 1 : 0;
    } else if (allow_pool) {
        size_t total = 0;
        for (int i = 0; i < n; ++i) {
            const DevJob& dj = r->host[i];
            total += (size_t)std::max(0, dj.cull[2] - dj.cull[0] + 1) * std::max(0, dj.cull[3] - dj.cull[1] + 1);
        }
        if (total > 0 && total * ray_record_bytes() < ((size_t)1 << 31) &&
            ensure_pool(ctx, total * ray_record_bytes(), stream)) {
            size_t off = 0;
            for (int i = 0; i < n; ++i) {
                DevJob& dj = r->host[i];
                dj.rays = static_cast<char*>(ctx->pool_rays) + off * ray_record_bytes();
                off += (size_t)std::max(0, dj.cull[2] - dj.cull[0] + 1) * std::max(0, dj.cull[3] - dj.cull[1] + 1);
            }
            la.dense_setup = 1;
        }
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (flags & ISAAC_TIMING) {
        t0 = get_event(ctx);
        t1 = get_event(ctx);
        if (!t0 || !t1) return set_err(ctx, ISAAC_ERR_DEVICE, "hipEventCreate failed");
    }
    const bool use_graph = n > 1 && !(flags & ISAAC_NO_GRAPH) && !noalloc;
    if (use_graph) {
        if (!r->exec || r->g_jobs != n || r->g_tiles != tiles || r->g_grid != la.grid || r->g_src != la.max_src ||
            r->g_unroll != la.unroll || r->g_lanes != la.lanes || r->g_hint != la.waves_hint || r->g_sig != la.sig ||
            r->g_fill != la.fill_blocks || r->g_dense != la.dense_setup) {
            if (r->exec) hipGraphExecDestroy(r->exec);
            if (r->graph) hipGraphDestroy(r->graph);
            r->exec = nullptr;
            r->graph = nullptr;
            HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipMemcpyAsync(r->dev, r->host, sizeof(DevJob) * n, hipMemcpyHostToDevice, ctx->cap_stream);
            if (e == hipSuccess) e = (hipError_t)launch_reset_counter(r->cursor, ctx->cap_stream);
            if (e == hipSuccess) e = (hipError_t)launch_prepass(la, ctx->cap_stream);
            if (e == hipSuccess) e = (hipError_t)launch_raycast(la, ctx->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return set_err(ctx, ISAAC_ERR_DEVICE, "graph capture failed: %s",
                               hipGetErrorString(e != hipSuccess ? e : e2));
            }
            r->graph = g;
            HIP_TRY(ctx, hipGraphInstantiate(&r->exec, g, nullptr, nullptr, 0));
            r->g_jobs = n;
            r->g_tiles = tiles;
            r->g_grid = la.grid;
            r->g_src = la.max_src;
            r->g_unroll = la.unroll;
            r->g_lanes = la.lanes;
            r->g_hint = la.waves_hint;
            r->g_sig = la.sig;
            r->g_fill = la.fill_blocks;
            r->g_dense = la.dense_setup;
        }
        if (t0) HIP_TRY(ctx, hipEventRecord(t0, stream));
        HIP_TRY(ctx, hipGraphLaunch(r->exec, stream));
        if (t1) HIP_TRY(ctx, hipEventRecord(t1, stream));
    } else if (n == 1 && allow_pool && !noalloc && djs[0].pool && lanes >= 2 && lanes <= 16 &&
               djs[0].mode == ISAAC_VOLUME &&
               (size_t)djs[0].width * djs[0].height * ray_record_bytes() < ((size_t)1 << 31) &&
               ensure_pool(ctx, (size_t)djs[0].width * djs[0].height * ray_record_bytes(), stream)) {
        // pooled schedule: compacted rays handed to lane groups as they free up
        HIP_TRY(ctx, hipMemcpyAsync(r->dev, r->host, sizeof(DevJob), hipMemcpyHostToDevice, stream));
        if (t0) HIP_TRY(ctx, hipEventRecord(t0, stream));
        int rc = launch_raycast_pooled(r->dev, djs[0].width, djs[0].height, ctx->tf_pool, la.max_src, la.sig, lanes,
                                       la.waves_hint, ctx->pool_rays, ctx->pool_counters, ctx->n_cu, stream);
        if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "raycast launch: %s", hipGetErrorString((hipError_t)rc));
        if (t1) HIP_TRY(ctx, hipEventRecord(t1, stream));
    } else {
        int rc = hipSuccess;
        if (n == 1 && !la.persistent) {
            // the job block travels as the prepass's kernel argument and is stored by it
            rc = launch_prepass_one(r->host[0], r->dev, la.fill_blocks, la.dense_setup, stream);
        } else {
            HIP_TRY(ctx, hipMemcpyAsync(r->dev, r->host, sizeof(DevJob) * n, hipMemcpyHostToDevice, stream));
            if (la.persistent) {
                rc = launch_reset_counter(r->cursor, stream);
                if (rc != hipSuccess)
                    return set_err(ctx, ISAAC_ERR_DEVICE, "counter reset: %s", hipGetErrorString((hipError_t)rc));
            }
            rc = launch_prepass(la, stream);
        }
        if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "prepass launch: %s", hipGetErrorString((hipError_t)rc));
        if (t0) HIP_TRY(ctx, hipEventRecord(t0, stream));
        rc = launch_raycast(la, stream);
        if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "raycast launch: %s", hipGetErrorString((hipError_t)rc));
        if (t1) HIP_TRY(ctx, hipEventRecord(t1, stream));
    }
    if (t0) ctx->timed.emplace_back(t0, t1);
    HIP_TRY(ctx, hipEventRecord(r->done, stream));
    r->busy = true;
    if (noalloc) {
        // the ring event: a later call re-records it only after waiting for it (acquire_slot),
        // so a query that sees newer work can only report this call's completion late
        ctx->pending.push_back({seq, r->done, false});
        return ISAAC_OK;
    }
    hipEvent_t pe = get_event(ctx);
    if (!pe) return set_err(ctx, ISAAC_ERR_DEVICE, "hipEventCreate failed");
    HIP_TRY(ctx, hipEventRecord(pe, stream));
    ctx->pending.push_back({seq, pe});
    return ISAAC_OK;
}

// Scan points a job is expected to take before clipping and termination:
// the volume's cells over the step, times the rays per cell cross-section at
// the volume's centre.
double estimate_samples(const DevJob& dj) {
    const double cells = (double)dj.dims[0] * dj.dims[1] * dj.dims[2];
    double px;   // pixels per voxel across the view at the volume centre
    if (dj.ortho) {
        px = dj.height / (2.0 * dj.h);
    } else {
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double c = dj.org[a] + 0.5 * dj.dims[a] - dj.eye[a];
            r2 += c * c;
        }
        px = dj.height / (2.0 * std::sqrt(std::max(r2, 1.0)) * dj.h);
    }
    return cells / dj.step * std::min(px * px, 1.0e6);
}

// Replace the sources of the call's jobs by derived volumes where that saves
// work: each voxel's chain output is then computed once per call instead of
// once per trilinear corner visit, and the ray loop gathers one interleaved
// FP32 value per source.  The values are the ones the loop would compute, so
// the image does not change.
isaac_status derive_volumes(isaac_context* ctx, const isaac_render_desc* jobs, std::vector<DevJob>& djs, bool force,
                            hipStream_t stream) {
    const int n = (int)djs.size();
    std::vector<int> vols;
    for (int i = 0; i < n; ++i)
        if (std::find(vols.begin(), vols.end(), jobs[i].volume_id) == vols.end()) vols.push_back(jobs[i].volume_id);
    for (int vid : vols) {
        Volume& v = ctx->volumes[vid];
        if (v.frozen) continue;       // its jobs already read the frozen derived volume
        int comp_of[kMaxSources];
        for (int s = 0; s < kMaxSources; ++s) comp_of[s] = -1;
        double est = 0.0;
        bool benefit = false;
        int g = 0;
        for (int i = 0; i < n; ++i) {
            if (jobs[i].volume_id != vid) continue;
            const DevJob& dj = djs[i];
            est += estimate_samples(dj) * (dj.interp ? 8.0 : 1.0);
            for (int k = 0; k < dj.n_src; ++k) {
                const DevSource& d = dj.src[k];
                comp_of[dj.src_index[k]] = 0;
                benefit = benefit || d.f_dim > 1 || d.n_ops > 0 || d.dtype != DT_F32 || !d.packed;
                g = std::max(g, (int)d.guard);
            }
        }
        int nd = 0;
        for (int s = 0; s < kMaxSources; ++s)
            if (comp_of[s] >= 0) comp_of[s] = nd++;
        if (nd == 0 || nd > kMaxDerived || !benefit) continue;
        const int64_t ex = v.dims[0] + 2 * g, ey = v.dims[1] + 2 * g, ez = v.dims[2] + 2 * g;
        // The derived sources in either layout: x fastest, or (three sources) the (y, z)
        // pairs, stored y and z shifted by gp, an even number of layers at least g, so
        // that index parity is the stored parity.
        const int gp = g + (g & 1);
        const int64_t ny2 = (ey - g + gp + 1) / 2, nz2 = (ez - g + gp + 1) / 2;
        struct Layout {
            bool paired;
            size_t bytes;
            int64_t sx, sy, sz, o0;
        };
        auto layout_of = [&](bool p) {
            Layout L;
            L.paired = p;
            if (p) {
                L.sx = 16 * nd;                         // 4 records per x
                L.sy = L.sx * ex;                       // per stored y pair
                L.sz = L.sy * ny2;                      // per stored z pair
                L.o0 = g * L.sx + (gp / 2) * (L.sy + L.sz);   // voxel (0, 0, 0): stored (g, gp, gp)
                L.bytes = (size_t)ex * ny2 * nz2 * 4 * nd * sizeof(float);
            } else {
                L.sx = 4 * nd;
                L.sy = L.sx * ex;
                L.sz = L.sy * ey;
                L.o0 = g * (L.sx + L.sy + L.sz);
                L.bytes = (size_t)ex * ey * ez * nd * sizeof(float);
            }
            return L;
        };
        auto describe = [&](DevJob& dj, const Layout& L, void* base) {
            for (int k = 0; k < dj.n_src; ++k) {
                DevSource& d = dj.src[k];
                const int guard = d.guard;
                std::memset(d.base, 0, sizeof d.base);
                std::memset(d.num_records, 0, sizeof d.num_records);
                std::memset(d.comp_off, 0, sizeof d.comp_off);
                d.base[0] = reinterpret_cast<uint64_t>(base);
                d.num_records[0] = (uint32_t)L.bytes;
                d.comp_off[0] = (int32_t)(L.o0 + 4 * comp_of[dj.src_index[k]]);
                d.packed = 1;
                d.layout = L.paired ? 1 : 0;
                d.stride[0] = (int32_t)L.sx;
                d.stride[1] = (int32_t)L.sy;
                d.stride[2] = (int32_t)L.sz;
                d.f_dim = 1;
                d.dtype = DT_F32;
                d.guard = guard;
                d.n_ops = 0;
            }
        };
        // The paired layout only when every job of the volume in this call then runs the
        // three-source loop, its only reader (calls with iso or fewer-source jobs keep x
        // fastest; a volume frozen in pairs is read directly by such jobs later).
        bool paired = nd == 3;
        if (paired) {
            const Layout P = layout_of(true);
            for (int i = 0; i < n && paired; ++i) {
                if (jobs[i].volume_id != vid) continue;
                DevJob t = djs[i];
                describe(t, P, reinterpret_cast<void*>((uintptr_t)256));
                paired = t.mode != ISAAC_ISO && signature_of(t) == SIG_IL3P;
            }
        }
        const Layout L = layout_of(paired);
        const size_t bytes = L.bytes;
        if (bytes >= ((size_t)1 << 31)) continue;
        if (!force && est < 4.0 * (double)(ex * ey * ez)) continue;
        if (v.derived_bytes != bytes) {
            if (v.derived) {
                HIP_TRY(ctx, hipStreamSynchronize(stream));
                HIP_TRY(ctx, hipFree(v.derived));
            }
            v.derived = nullptr;
            v.derived_bytes = 0;
            if (hipMalloc(&v.derived, bytes) != hipSuccess) {
                v.derived = nullptr;
                continue;             // no memory: read the sources directly
            }
            v.derived_bytes = bytes;
        }
        // the sources as the ray loop would read them, from the first job using each
        DeriveArgs da;
        std::memset(&da, 0, sizeof da);
        da.n = nd;
        da.g = g;
        da.ext[0] = (int)ex;
        da.ext[1] = (int)ey;
        da.ext[2] = (int)ez;
        da.paired = paired ? 1 : 0;
        da.gp = gp;
        da.ny2 = (int)ny2;
        da.nz2 = (int)nz2;
        da.dst = static_cast<float*>(v.derived);
        for (int i = 0; i < n; ++i) {
            if (jobs[i].volume_id != vid) continue;
            for (int k = 0; k < djs[i].n_src; ++k) da.src[comp_of[djs[i].src_index[k]]] = djs[i].src[k];
        }
        // voxels clipped away for every job of the volume are never read: skip them
        // (up to kMaxKeepSets jobs; a job without planes needs every voxel)
        int sets = 0;
        bool all_voxels = false;
        for (int i = 0; i < n && !all_voxels; ++i) {
            if (jobs[i].volume_id != vid) continue;
            const DevJob& dj = djs[i];
            bool same_org = true;
            for (int i0 = 0; i0 < i; ++i0)
                if (jobs[i0].volume_id == vid)
                    for (int a = 0; a < 3; ++a) same_org = same_org && djs[i0].org[a] == dj.org[a];
            if (dj.n_clip == 0 || sets == kMaxKeepSets || !same_org) {
                all_voxels = true;
                break;
            }
            da.n_planes[sets] = dj.n_clip;
            for (int c = 0; c < dj.n_clip; ++c) {
                const double* pl = dj.clip[c];
                const double nl = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
                for (int e = 0; e < 4; ++e) da.planes[sets][c][e] = (float)(pl[e] / nl);
            }
            ++sets;
        }
        da.n_sets = all_voxels ? 0 : sets;
        for (int a = 0; a < 3; ++a) da.org[a] = djs[0].org[a];
        for (int i = 0; i < n; ++i)
            if (jobs[i].volume_id == vid) {
                for (int a = 0; a < 3; ++a) da.org[a] = djs[i].org[a];
                break;
            }
        // the sources' own signature selects a compile-time specialized derive
        DevJob probe;
        std::memset(&probe, 0, sizeof probe);
        probe.n_src = nd;
        for (int k = 0; k < nd; ++k) probe.src[k] = da.src[k];
        const int dsig = signature_of(probe);
        int rc = launch_derive(da, dsig == SIG_IL3 || dsig == SIG_IL3P ? (int)SIG_GENERIC : dsig, stream);
        if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "derive launch: %s", hipGetErrorString((hipError_t)rc));
        for (int i = 0; i < n; ++i) {
            if (jobs[i].volume_id != vid) continue;
            DevJob& dj = djs[i];
            describe(dj, L, v.derived);
            if (dj.mode != ISAAC_ISO) dj.sig = signature_of(dj);
        }
    }
    return ISAAC_OK;
}

isaac_status render_impl(isaac_context* ctx, const isaac_render_desc* jobs, int n, unsigned flags, bool need_out,
                         hipStream_t stream, bool allow_derive, bool noalloc = false) {
    if (n < 1 || n > kMaxBatch || !jobs)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "n_jobs must be 1..%d", kMaxBatch);
    std::vector<DevJob> djs(n);
    int max_src = 1;
    for (int i = 0; i < n; ++i) {
        int na = 0;
        isaac_status st = build_job(ctx, jobs[i], need_out, djs[i], &na);
        if (st) return st;
        max_src = std::max(max_src, na);
    }
    if (noalloc) {
        // every job's ray records must fit the scratch together (checked before any update())
        size_t rays = 0;
        for (const DevJob& dj : djs)
            rays += (size_t)std::max(0, dj.cull[2] - dj.cull[0] + 1) * std::max(0, dj.cull[3] - dj.cull[1] + 1);
        if (rays * ray_record_bytes() > kNoAllocScratchBytes)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT,
                           "the jobs' screen rectangles need %zu ray records of %zu bytes, above the %zu-byte "
                           "scratch of calls that allocate nothing", rays, ray_record_bytes(), kNoAllocScratchBytes);
    }
    isaac_status st = prepare_sources(ctx, jobs, n);
    if (st) return st;
    // non-persistent sources read their shadow copies
    for (int i = 0; i < n; ++i) {
        const Volume& v = ctx->volumes[jobs[i].volume_id];
        for (int k = 0; k < djs[i].n_src; ++k) {
            const SourceHost& sh = v.src[djs[i].src_index[k]];
            if (!sh.desc.persistent) {
                DevSource& ds = djs[i].src[k];
                const int es = esize_of(sh.desc.dtype);
                const int64_t ex = v.dims[0] + 2 * sh.reach, ey = v.dims[1] + 2 * sh.reach;
                ds.base[0] = reinterpret_cast<uint64_t>(sh.shadow);
                ds.num_records[0] = (uint32_t)sh.shadow_bytes;
                ds.stride[0] = sh.desc.f_dim * es;
                ds.stride[1] = (int32_t)(sh.desc.f_dim * es * ex);
                ds.stride[2] = (int32_t)(sh.desc.f_dim * es * ex * ey);
                const int32_t o = sh.reach * (ds.stride[0] + ds.stride[1] + ds.stride[2]);
                for (int c = 0; c < 4; ++c) ds.comp_off[c] = o + c * es;
                ds.packed = 1;
            }
        }
    }
    // frozen volumes: every job reads the derived values (render and serving calls
    // alike), except, on a volume frozen in (y, z) pairs, a job that would not run
    // the three-source loop (the layout's only reader): it reads the unchanged
    // sources directly
    for (int i = 0; i < n; ++i) {
        const Volume& v = ctx->volumes[jobs[i].volume_id];
        if (!v.frozen || (flags & ISAAC_DIRECT)) continue;
        DevJob& dj = djs[i];
        DevJob t = dj;
        for (int k = 0; k < t.n_src; ++k) {
            const DevSource& f = v.frozen_src[t.src_index[k]];
            DevSource& d = t.src[k];
            std::memcpy(d.base, f.base, sizeof d.base);
            std::memcpy(d.num_records, f.num_records, sizeof d.num_records);
            std::memcpy(d.comp_off, f.comp_off, sizeof d.comp_off);
            std::memcpy(d.stride, f.stride, sizeof d.stride);
            d.packed = f.packed;
            d.layout = f.layout;
            d.f_dim = 1;
            d.dtype = DT_F32;
            d.n_ops = 0;
        }
        if (t.mode != ISAAC_ISO) t.sig = signature_of(t);
        const bool paired = t.n_src > 0 && t.src[0].layout == 1;
        if (!paired || (t.mode != ISAAC_ISO && t.sig == SIG_IL3P)) dj = t;
    }
    if (allow_derive && !(flags & ISAAC_DIRECT)) {
        st = derive_volumes(ctx, jobs, djs, (flags & ISAAC_DERIVE) != 0, stream);
        if (st) return st;
    }
    // one launch per scan-point schedule, so every job is rendered exactly as
    // it would be alone (its size class's lanes per ray, unroll and variant)
    std::vector<std::vector<DevJob>> groups;
    std::vector<int> keys;
    for (const DevJob& dj : djs) {
        const int key = dj.mode * 2048 + dj.pool * 1024 + dj.lanes * 16 + dj.unroll * 2 + dj.waves_hint;
        size_t g = 0;
        while (g < keys.size() && keys[g] != key) ++g;
        if (g == keys.size()) {
            keys.push_back(key);
            groups.emplace_back();
        }
        groups[g].push_back(dj);
    }
    for (const auto& grp : groups) {
        int ms = 1;
        for (const DevJob& dj : grp) ms = std::max(ms, (int)dj.n_src);
        st = enqueue_jobs(ctx, jobs, grp, ms, flags, stream, allow_derive, noalloc);
        if (st) return st;
    }
    (void)max_src;
    if (!(flags & ISAAC_ASYNC)) {
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        update_completed(ctx);
    }
    return ISAAC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* isaac_version(void) { return "isaac-mi355x 0.1 (gfx950)"; }

const char* isaac_init_error(void) { return g_init_error.c_str(); }

const char* isaac_last_error(const isaac_context* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

isaac_status isaac_check_functor_chain(const char* chain, int f_dim, int* out_dim, int* out_ops, char* err,
                                       int errlen) {
    CompiledChain c;
    std::string e;
    if (!compile_chain(chain, f_dim, c, e)) {
        if (err && errlen > 0) std::snprintf(err, (size_t)errlen, "%s", e.c_str());
        return ISAAC_ERR_BAD_FUNCTOR;
    }
    if (out_dim) *out_dim = c.out_dim;
    if (out_ops) *out_ops = c.n_ops;
    if (err && errlen > 0) err[0] = 0;
    return ISAAC_OK;
}

isaac_status isaac_init(const isaac_init_desc* desc, isaac_context** out) {
    if (!out) return ISAAC_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    isaac_init_desc d{};
    if (desc) d = *desc;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev < 1) {
        g_init_error = "no HIP device";
        return ISAAC_ERR_DEVICE;
    }
    if (d.device < 0 || d.device >= n_dev) {
        g_init_error = "device ordinal out of range";
        return ISAAC_ERR_INVALID_ARGUMENT;
    }
    if (d.flags & ~ISAAC_INIT_NULL_STREAM) {
        g_init_error = "unknown isaac_init_desc.flags bits";
        return ISAAC_ERR_INVALID_ARGUMENT;
    }
    if (d.stream && (d.flags & ISAAC_INIT_NULL_STREAM)) {
        g_init_error = "ISAAC_INIT_NULL_STREAM needs stream == NULL";
        return ISAAC_ERR_INVALID_ARGUMENT;
    }
    auto* ctx = new isaac_context();
    ctx->device = d.device;
    ctx->budget = d.mem_budget_bytes ? d.mem_budget_bytes : ((size_t)1 << 30);
    ctx->max_inflight = d.max_inflight > 0 ? d.max_inflight : 64;
    ctx->volumes.resize(d.max_volumes > 0 ? d.max_volumes : 256);
    auto fail = [&](const char* what, hipError_t e) {
        g_init_error = std::string(what) + ": " + hipGetErrorString(e);
        isaac_destroy(ctx);
        return ISAAC_ERR_DEVICE;
    };
    hipError_t e = hipSetDevice(d.device);
    if (e != hipSuccess) return fail("hipSetDevice", e);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, d.device);
    if (e != hipSuccess) return fail("hipGetDeviceProperties", e);
    ctx->n_cu = prop.multiProcessorCount;
    {
        const int rc = noalloc_scratch(d.device, &ctx->noalloc_scratch);   // d.device is current
        if (rc != hipSuccess) return fail("scratch symbol address", (hipError_t)rc);
    }
    int bpc = 1;
    if (raycast_occupancy(&bpc) == hipSuccess && bpc > 0) ctx->blocks_per_cu = bpc;
    if (d.stream) {
        ctx->stream = static_cast<hipStream_t>(d.stream);
    } else if (d.flags & ISAAC_INIT_NULL_STREAM) {
        ctx->stream = nullptr;                  // the null stream, borrowed like any caller stream
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail("hipStreamCreate", e);
        ctx->own_stream = true;
    }
    e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail("hipStreamCreate", e);
    for (int i = 0; i < 4; ++i) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return fail("hipStreamCreate", e);
        ctx->serve_streams.push_back(s);
    }
    for (int i = 0; i < kRingSlots; ++i) {
        RingSlot& r = ctx->ring[i];
        e = hipHostMalloc((void**)&r.host, sizeof(DevJob) * kMaxBatch);
        if (e == hipSuccess) e = hipMalloc((void**)&r.dev, sizeof(DevJob) * kMaxBatch);
        if (e == hipSuccess) e = hipMalloc((void**)&r.cursor, 64);
        if (e == hipSuccess) e = hipMemset(r.cursor, 0, 64);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
        if (e != hipSuccess) return fail("staging ring", e);
    }
    e = hipMalloc((void**)&ctx->tf_pool, (size_t)kTfSlots * kTfRows * 4 * sizeof(float));
    if (e != hipSuccess) return fail("transfer table pool", e);
    ctx->tf_capacity = kTfSlots;
    ctx->tf_slots.resize(kTfSlots);
    // slot 0: the all-zero table of sources without a transfer function
    e = hipMemset(ctx->tf_pool, 0, kTfRows * 4 * sizeof(float));
    if (e != hipSuccess) return fail("hipMemset", e);
    ctx->tf_slots[0].live = true;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail("hipDeviceSynchronize", e);
    *out = ctx;
    return ISAAC_OK;
}

void isaac_destroy(isaac_context* ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (hipStream_t s : ctx->serve_streams) hipStreamSynchronize(s);
    hipDeviceSynchronize();
    for (auto& v : ctx->volumes) {
        for (auto& s : v.src)
            if (s.shadow) hipFree(s.shadow);
        if (v.derived) hipFree(v.derived);
    }
    for (auto& kv : ctx->tickets) {
        if (kv.second.out) hipFree(kv.second.out);
        if (kv.second.ev) hipEventDestroy(kv.second.ev);
    }
    ctx->images.destroy();
    for (auto& r : ctx->ring) {
        if (r.exec) hipGraphExecDestroy(r.exec);
        if (r.graph) hipGraphDestroy(r.graph);
        if (r.host) hipHostFree(r.host);
        if (r.dev) hipFree(r.dev);
        if (r.cursor) hipFree(r.cursor);
        if (r.done) hipEventDestroy(r.done);
    }
    for (auto& p : ctx->pending) hipEventDestroy(p.ev);
    for (auto& t : ctx->timed) {
        hipEventDestroy(t.first);
        hipEventDestroy(t.second);
    }
    for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
    if (ctx->tf_pool) hipFree(ctx->tf_pool);
    if (ctx->enc_buf) hipFree(ctx->enc_buf);
    isaac::jpeg_work_destroy(ctx->jpeg);
    if (ctx->pool_rays) hipFree(ctx->pool_rays);
    if (ctx->pool_counters) hipFree(ctx->pool_counters);
    for (hipStream_t s : ctx->serve_streams) hipStreamDestroy(s);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
    delete ctx;
}

isaac_status isaac_set_sources(isaac_context* ctx, int volume_id, const int32_t dims[3], const isaac_source_desc* src,
                               int n_src) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (volume_id < 0 || volume_id >= (int)ctx->volumes.size())
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "volume id %d outside 0..%d", volume_id, (int)ctx->volumes.size() - 1);
    if (!dims) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "dims is NULL");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > (1 << 20))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "dims[%d] = %d outside 1..2^20", a, dims[a]);
    if (n_src < 0 || n_src > kMaxSources || (n_src > 0 && !src))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "n_src must be 0..%d", kMaxSources);
    std::vector<SourceHost> hs(n_src);
    for (int s = 0; s < n_src; ++s) {
        SourceHost& h = hs[s];
        h.desc = src[s];
        h.name = src[s].name ? src[s].name : ("source" + std::to_string(s));
        h.chain_text = src[s].functor_chain ? src[s].functor_chain : "";
        h.desc.name = nullptr;
        h.desc.functor_chain = nullptr;
        const isaac_source_desc& d = src[s];
        if (d.f_dim < 1 || d.f_dim > 4)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': f_dim %d outside 1..4", h.name.c_str(), d.f_dim);
        if (d.dtype != ISAAC_F32 && d.dtype != ISAAC_F16 && d.dtype != ISAAC_BF16)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': unknown dtype", h.name.c_str());
        if (d.guard < 0) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': guard < 0", h.name.c_str());
        if (!(d.weight >= 0.0f && d.weight <= 1.0f))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': weight must lie in [0,1]", h.name.c_str());
        std::string err;
        if (!compile_chain(h.chain_text.c_str(), d.f_dim, h.chain, err))
            return set_err(ctx, ISAAC_ERR_BAD_FUNCTOR, "source '%s': %s", h.name.c_str(), err.c_str());
        const int es = esize_of(d.dtype);
        bool have = true;
        for (int c = 0; c < d.f_dim; ++c) have = have && d.comp[c] != nullptr;
        if (!have) {
            if (d.enabled)
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': enabled with a NULL component",
                               h.name.c_str());
            h.desc.comp[0] = nullptr;   // never read
            continue;
        }
        for (int c = 0; c < d.f_dim; ++c)
            if (reinterpret_cast<uintptr_t>(d.comp[c]) % es)
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': component %d misaligned", h.name.c_str(), c);
        for (int a = 0; a < 3; ++a)
            if (d.stride[a] % es)
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source '%s': stride %d not a multiple of %d bytes",
                               h.name.c_str(), a, es);
        st = derive_layout(ctx, dims, h);
        if (st) return st;
    }
    // allocate shadows for non-persistent sources (all or nothing)
    for (int s = 0; s < n_src; ++s) {
        SourceHost& h = hs[s];
        if (h.desc.persistent || !h.desc.comp[0]) continue;
        const int reach = h.desc.guard >= 1 ? 1 : 0;
        h.shadow_bytes = (size_t)esize_of(h.desc.dtype) * h.desc.f_dim * (dims[0] + 2 * reach) *
                         (size_t)(dims[1] + 2 * reach) * (dims[2] + 2 * reach);
        if (h.shadow_bytes >= ((size_t)1 << 31)) {
            for (auto& x : hs)
                if (x.shadow) hipFree(x.shadow);
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "non-persistent source '%s' larger than 2 GiB",
                           h.name.c_str());
        }
        if (hipMalloc(&h.shadow, h.shadow_bytes) != hipSuccess) {
            for (auto& x : hs)
                if (x.shadow) hipFree(x.shadow);
            return set_err(ctx, ISAAC_ERR_OUT_OF_MEMORY, "no memory for the copy of source '%s'", h.name.c_str());
        }
    }
    Volume& v = ctx->volumes[volume_id];
    if (v.defined) {
        hipStreamSynchronize(ctx->stream);
        for (auto& s : v.src)
            if (s.shadow) hipFree(s.shadow);
        if (v.derived) hipFree(v.derived);
        v.derived = nullptr;
        v.derived_bytes = 0;
    }
    v.frozen = false;
    std::vector<int32_t> tf(n_src, 0);
    for (int s = 0; s < n_src && s < (int)v.tf.size(); ++s) tf[s] = v.tf[s];
    v.defined = true;
    for (int a = 0; a < 3; ++a) v.dims[a] = dims[a];
    v.src = std::move(hs);
    v.tf = tf;
    return ISAAC_OK;
}

isaac_status isaac_set_transfer(isaac_context* ctx, int volume_id, int source, const isaac_tf_point* pts, int n_pts,
                                int32_t* out_handle) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (volume_id < 0 || volume_id >= (int)ctx->volumes.size() || !ctx->volumes[volume_id].defined)
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "volume %d is not defined", volume_id);
    Volume& v = ctx->volumes[volume_id];
    if (source < 0 || source >= (int)v.src.size())
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "volume %d has no source %d", volume_id, source);
    float table[kTfEntries * 4];
    std::string err;
    if (!bake_tf(pts, n_pts, table, err)) return set_err(ctx, ISAAC_ERR_BAD_TRANSFER, "%s", err.c_str());
    int32_t h = -1;
    st = new_tf_slot(ctx, table, &h);
    if (st) return st;
    v.tf[source] = h;
    if (out_handle) *out_handle = h;
    return ISAAC_OK;
}

isaac_status isaac_release_transfer(isaac_context* ctx, int32_t handle) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (handle <= 0 || handle >= ctx->tf_capacity || !ctx->tf_slots[handle].live || ctx->tf_slots[handle].released)
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "transfer handle %d is not live", handle);
    ctx->tf_slots[handle].released = true;   // a current table stays until replaced
    update_completed(ctx);
    return ISAAC_OK;
}

isaac_status isaac_render(isaac_context* ctx, const isaac_render_desc* jobs, int n_jobs, unsigned flags) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    return render_impl(ctx, jobs, n_jobs, flags, true, ctx->stream, true);
}

isaac_status isaac_render_noalloc(isaac_context* ctx, const isaac_render_desc* jobs, int n_jobs, unsigned flags) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (flags & ~(ISAAC_ASYNC | ISAAC_NO_GRAPH | ISAAC_DIRECT))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT,
                       "isaac_render_noalloc takes ISAAC_ASYNC, ISAAC_NO_GRAPH and ISAAC_DIRECT only");
    if (!ctx->noalloc_scratch) return set_err(ctx, ISAAC_ERR_DEVICE, "no scratch address for this device");
    return render_impl(ctx, jobs, n_jobs, flags | ISAAC_NO_GRAPH, true, ctx->stream, false, true);
}

isaac_status isaac_composite(isaac_context* ctx, const float* const* rgba, const float* const* depth, int n_layers,
                             int width, int height, float* out, unsigned flags) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (n_layers < 1 || n_layers > kMaxLayers || !rgba || !depth || !out || width < 1 || height < 1)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "composite needs 1..%d layers, pointers and a size", kMaxLayers);
    for (int l = 0; l < n_layers; ++l) {
        if (!rgba[l] || !depth[l]) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "layer %d has a NULL pointer", l);
        if (!aligned_to(rgba[l], 16) || !aligned_to(depth[l], 4))
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "layer %d: rgba must be 16-byte, depth 4-byte aligned", l);
    }
    if (!aligned_to(out, 16)) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "out must be 16-byte aligned");
    int rc = launch_composite(rgba, depth, n_layers, (int64_t)width * height, out, ctx->stream);
    if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "composite launch: %s", hipGetErrorString((hipError_t)rc));
    if (!(flags & ISAAC_ASYNC)) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return ISAAC_OK;
}

isaac_status isaac_encode_rgba8(isaac_context* ctx, const float* rgba, int width, int height, const float* background,
                                unsigned char* out, unsigned flags) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (!rgba || !out || width < 1 || height < 1)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "encode needs an image, an output and a size");
    if (!aligned_to(rgba, 16) || !aligned_to(out, 4))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "rgba must be 16-byte and out 4-byte aligned");
    if (background)
        for (int c = 0; c < 3; ++c)
            if (!(background[c] >= 0.f && background[c] <= 1.f))
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "background channel %d must lie in [0,1]", c);
    int rc = launch_encode_rgba8(rgba, (int64_t)width * height, background, out, ctx->stream);
    if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "encode launch: %s", hipGetErrorString((hipError_t)rc));
    if (!(flags & ISAAC_ASYNC)) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return ISAAC_OK;
}

isaac_status isaac_freeze_volume(isaac_context* ctx, int volume_id) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (volume_id < 0 || volume_id >= (int)ctx->volumes.size() || !ctx->volumes[volume_id].defined)
        return set_err(ctx, ISAAC_ERR_NOT_FOUND, "volume %d is not defined", volume_id);
    Volume& v = ctx->volumes[volume_id];
    if (v.frozen) return ISAAC_OK;
    const int ns = (int)v.src.size();
    if (ns < 1 || ns > kMaxDerived)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "a frozen volume has 1..%d sources", kMaxDerived);
    for (int s = 0; s < ns; ++s) {
        if (!v.src[s].desc.persistent)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source %d is not persistent: it cannot be frozen", s);
        if (!v.src[s].desc.comp[0]) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "source %d has no data", s);
    }
    // a job that reads every source: one pixel, orthographic, no clip planes
    isaac_render_desc d;
    std::memset(&d, 0, sizeof d);
    d.volume_id = volume_id;
    d.width = d.height = 1;
    d.projection = ISAAC_ORTHOGRAPHIC;
    for (int a = 0; a < 3; ++a) d.center[a] = 0.5 * v.dims[a];
    d.eye[0] = d.center[0] - v.dims[0] - 1.0;
    d.eye[1] = d.center[1];
    d.eye[2] = d.center[2];
    d.up[2] = 1.0;
    d.ortho_height = 1.0;
    d.step = 1.0;
    d.interpolation = ISAAC_TRILINEAR;
    int32_t en[kMaxSources];
    float w[kMaxSources];
    for (int s = 0; s < ns; ++s) en[s] = 1, w[s] = 1.0f;
    d.enabled = en;
    d.weights = w;
    std::vector<DevJob> djs(1);
    int na = 0;
    st = build_job(ctx, d, false, djs[0], &na);
    if (st) return st;
    st = prepare_sources(ctx, &d, 1);
    if (st) return st;
    st = derive_volumes(ctx, &d, djs, true, ctx->stream);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const DevJob& dj = djs[0];
    if (dj.n_src != ns || !v.derived || dj.src[0].base[0] != reinterpret_cast<uint64_t>(v.derived))
        return ISAAC_OK;   // the sources are read directly already (plain FP32 scalars) or no memory: nothing to freeze
    for (int k = 0; k < dj.n_src; ++k) v.frozen_src[dj.src_index[k]] = dj.src[k];
    v.frozen = true;
    return ISAAC_OK;
}

isaac_status isaac_encode_jpeg(isaac_context* ctx, const unsigned char* rgba8, int width, int height, int quality,
                               unsigned char* out, size_t capacity, size_t* out_size) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (rgba8 && !aligned_to(rgba8, 4)) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "rgba8 must be 4-byte aligned");
    if (!ctx->jpeg) ctx->jpeg = isaac::jpeg_work_create();
    char msg[256] = {0};
    const int rc = isaac::jpeg_encode(ctx->jpeg, rgba8, width, height, quality, ctx->stream, out, capacity, out_size,
                                      msg, sizeof msg);
    if (rc) return set_err(ctx, (isaac_status)rc, "jpeg: %s", msg);
    return ISAAC_OK;
}

isaac_status isaac_timing(isaac_context* ctx, double* total_ms, int* count) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    double sum = 0.0;
    int n = 0;
    for (auto& t : ctx->timed) {
        HIP_TRY(ctx, hipEventSynchronize(t.second));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, t.first, t.second));
        sum += ms;
        ++n;
        put_event(ctx, t.first);
        put_event(ctx, t.second);
    }
    ctx->timed.clear();
    if (total_ms) *total_ms = sum;
    if (count) *count = n;
    return ISAAC_OK;
}

isaac_status isaac_set_tile_shape(isaac_context* ctx, int size_class, int wave_w, int waves_x, int unroll,
                                  int lanes_per_ray, int min_waves, int pooled) {
    if (!ctx) return ISAAC_ERR_INVALID_ARGUMENT;
    const int g = lanes_per_ray;
    const bool lanes_ok = g == 1 || g == 2 || g == 4 || g == 8 || g == 16 || g == 32 || g == 64;
    const bool ww_ok = wave_w >= 1 && wave_w <= 64 && (wave_w & (wave_w - 1)) == 0 && lanes_ok && wave_w <= 64 / g;
    if (size_class < 0 || size_class > 15 || !ww_ok || (waves_x != 1 && waves_x != 2 && waves_x != 4) ||
        (unroll != 1 && unroll != 2) || (g > 1 && unroll != 1) || (min_waves != 0 && min_waves != 4) ||
        (min_waves == 4 && (g == 2 || g >= 32 || unroll == 2)) || (pooled != 0 && pooled != 1) ||
        (pooled == 1 && (g < 2 || g > 16)))
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "invalid tile shape");
    ctx->shapes[size_class] = TileShape{wave_w, waves_x, unroll, g, min_waves == 4 ? 1 : 0, pooled};
    return ISAAC_OK;
}

isaac_status isaac_get_tile_shape(isaac_context* ctx, int size_class, int* wave_w, int* waves_x, int* unroll,
                                  int* lanes_per_ray, int* min_waves, int* pooled) {
    if (!ctx || size_class < 0 || size_class > 15) return ISAAC_ERR_INVALID_ARGUMENT;
    const TileShape& t = ctx->shapes[size_class];
    if (wave_w) *wave_w = t.wave_w;
    if (waves_x) *waves_x = t.waves_x;
    if (unroll) *unroll = t.unroll;
    if (lanes_per_ray) *lanes_per_ray = t.lanes;
    if (min_waves) *min_waves = t.waves_hint ? 4 : 0;
    if (pooled) *pooled = t.pool;
    return ISAAC_OK;
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------
isaac_status isaac_submit_batch(isaac_context* ctx, const isaac_render_desc* jobs, int n, uint64_t* tickets) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    if (n < 1 || n > kMaxBatch || !jobs || !tickets)
        return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "n_jobs must be 1..%d with a ticket array", kMaxBatch);
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        if (jobs[i].width < 1 || jobs[i].height < 1 || jobs[i].width > 32768 || jobs[i].height > 32768)
            return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "image size out of range");
        need += ImageArena::rounded((size_t)jobs[i].width * jobs[i].height * 4 * sizeof(float));
    }
    size_t inflight = ctx->tickets.size();
    if ((int)(inflight + n) > ctx->max_inflight || ctx->used + need > ctx->budget)
        return set_err(ctx, ISAAC_ERR_BUSY, "admission refused: %zu + %zu bytes of %zu, %zu in flight", ctx->used, need,
                       ctx->budget, inflight);
    // validate before allocating anything
    std::vector<isaac_render_desc> js(jobs, jobs + n);
    for (int i = 0; i < n; ++i) {
        DevJob tmp;
        int na = 0;
        js[i].out_rgba = reinterpret_cast<float*>(16);   // placeholder for validation only
        js[i].out_samples = nullptr;
        st = build_job(ctx, js[i], true, tmp, &na);
        if (st) return st;
    }
    if (!ctx->images.ready() && !ctx->images.init(ctx->budget))
        return set_err(ctx, ISAAC_ERR_OUT_OF_MEMORY, "no device memory for the %zu-byte serving budget", ctx->budget);
    std::vector<Ticket> made;
    auto give_back = [&]() {
        for (auto& m : made) ctx->images.give(m.out, m.bytes);
    };
    for (int i = 0; i < n; ++i) {
        Ticket t;
        t.bytes = (size_t)jobs[i].width * jobs[i].height * 4 * sizeof(float);   // the image (the arena rounds)
        t.width = jobs[i].width;
        t.height = jobs[i].height;
        t.out = ctx->images.take(t.bytes);
        if (!t.out) {
            give_back();
            return set_err(ctx, ISAAC_ERR_BUSY, "admission refused: no free run of %zu bytes in the budget "
                           "(%zu of %zu bytes in use)", t.bytes, ctx->used, ctx->budget);
        }
        js[i].out_rgba = t.out;
        made.push_back(t);
    }
    std::vector<hipEvent_t> evs(n, nullptr);
    for (int i = 0; i < n; ++i)
        if (!(evs[i] = get_event(ctx))) {
            for (hipEvent_t e : evs) put_event(ctx, e);
            give_back();
            return set_err(ctx, ISAAC_ERR_DEVICE, "hipEventCreate failed");
        }
    hipStream_t s = ctx->serve_streams[ctx->serve_rr];
    ctx->serve_rr = (ctx->serve_rr + 1) % (int)ctx->serve_streams.size();
    st = render_impl(ctx, js.data(), n, ISAAC_ASYNC | ISAAC_NO_GRAPH, true, s, false);
    if (st) {
        for (hipEvent_t e : evs) put_event(ctx, e);
        give_back();
        return st;
    }
    for (int i = 0; i < n; ++i) {
        Ticket& t = made[i];
        t.id = ctx->next_ticket++;
        t.ev = evs[i];
        HIP_TRY(ctx, hipEventRecord(t.ev, s));
        ctx->used += ImageArena::rounded(t.bytes);
        tickets[i] = t.id;
        ctx->tickets[t.id] = t;
    }
    return ISAAC_OK;
}

isaac_status isaac_submit(isaac_context* ctx, const isaac_render_desc* job, uint64_t* out_ticket) {
    return isaac_submit_batch(ctx, job, 1, out_ticket);
}

isaac_status isaac_poll(isaac_context* ctx, uint64_t ticket, int* done, const float** out_rgba) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return set_err(ctx, ISAAC_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket& t = it->second;
    if (!t.done) {
        hipError_t e = hipEventQuery(t.ev);
        if (e == hipSuccess) t.done = true;
        else if (e != hipErrorNotReady) return set_err(ctx, ISAAC_ERR_DEVICE, "request failed: %s", hipGetErrorString(e));
    }
    if (done) *done = t.done ? 1 : 0;
    if (out_rgba) *out_rgba = t.done ? t.out : nullptr;
    return ISAAC_OK;
}

isaac_status isaac_release(isaac_context* ctx, uint64_t ticket) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return set_err(ctx, ISAAC_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket& t = it->second;
    if (!t.done) HIP_TRY(ctx, hipEventSynchronize(t.ev));
    put_event(ctx, t.ev);
    ctx->used -= ImageArena::rounded(t.bytes);
    ctx->images.give(t.out, t.bytes);
    ctx->tickets.erase(it);
    update_completed(ctx);
    return ISAAC_OK;
}

isaac_status isaac_read_image(isaac_context* ctx, uint64_t ticket, float* host_rgba) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return set_err(ctx, ISAAC_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!host_rgba) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "host_rgba is NULL");
    Ticket& t = it->second;
    HIP_TRY(ctx, hipEventSynchronize(t.ev));
    t.done = true;
    HIP_TRY(ctx, hipMemcpy(host_rgba, t.out, t.bytes, hipMemcpyDeviceToHost));
    return ISAAC_OK;
}

isaac_status isaac_read_image_rgba8(isaac_context* ctx, uint64_t ticket, const float* background,
                                    unsigned char* host_rgba8) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return set_err(ctx, ISAAC_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!host_rgba8) return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "host_rgba8 is NULL");
    if (background)
        for (int c = 0; c < 3; ++c)
            if (!(background[c] >= 0.f && background[c] <= 1.f))
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "background channel %d must lie in [0,1]", c);
    Ticket& t = it->second;
    const int64_t n = (int64_t)(t.bytes / 16);
    if ((size_t)n * 4 > ctx->enc_bytes) {
        if (ctx->enc_buf) HIP_TRY(ctx, hipFree(ctx->enc_buf));
        ctx->enc_buf = nullptr;
        ctx->enc_bytes = 0;
        HIP_TRY(ctx, hipMalloc(&ctx->enc_buf, (size_t)n * 4));
        ctx->enc_bytes = (size_t)n * 4;
    }
    // encode after the render on the context stream, then copy 4 bytes per pixel
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, t.ev, 0));
    int rc = launch_encode_rgba8(t.out, n, background, static_cast<unsigned char*>(ctx->enc_buf), ctx->stream);
    if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "encode launch: %s", hipGetErrorString((hipError_t)rc));
    HIP_TRY(ctx, hipMemcpyAsync(host_rgba8, ctx->enc_buf, (size_t)n * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    t.done = true;
    return ISAAC_OK;
}

isaac_status isaac_read_image_jpeg(isaac_context* ctx, uint64_t ticket, const float* background, int quality,
                                   unsigned char* out, size_t capacity, size_t* out_size) {
    isaac_status st = check_ctx(ctx);
    if (st) return st;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return set_err(ctx, ISAAC_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (background)
        for (int c = 0; c < 3; ++c)
            if (!(background[c] >= 0.f && background[c] <= 1.f))
                return set_err(ctx, ISAAC_ERR_INVALID_ARGUMENT, "background channel %d must lie in [0,1]", c);
    Ticket& t = it->second;
    const int64_t n = (int64_t)(t.bytes / 16);
    if ((size_t)n * 4 > ctx->enc_bytes) {
        if (ctx->enc_buf) HIP_TRY(ctx, hipFree(ctx->enc_buf));
        ctx->enc_buf = nullptr;
        ctx->enc_bytes = 0;
        HIP_TRY(ctx, hipMalloc(&ctx->enc_buf, (size_t)n * 4));
        ctx->enc_bytes = (size_t)n * 4;
    }
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, t.ev, 0));
    int rc = launch_encode_rgba8(t.out, n, background, static_cast<unsigned char*>(ctx->enc_buf), ctx->stream);
    if (rc != hipSuccess) return set_err(ctx, ISAAC_ERR_DEVICE, "encode launch: %s", hipGetErrorString((hipError_t)rc));
    st = isaac_encode_jpeg(ctx, static_cast<const unsigned char*>(ctx->enc_buf), t.width, t.height, quality, out,
                           capacity, out_size);
    if (st == ISAAC_OK) t.done = true;
    return st;
}

isaac_status isaac_serving_usage(isaac_context* ctx, size_t* used, size_t* budget, int* inflight) {
    if (!ctx) return ISAAC_ERR_INVALID_ARGUMENT;
    if (used) *used = ctx->used;
    if (budget) *budget = ctx->budget;
    if (inflight) *inflight = (int)ctx->tickets.size();
    return ISAAC_OK;
}

}  // extern "C"
