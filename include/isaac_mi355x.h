/*
 * isaac_mi355x.h -- C ABI of an MI355X (gfx950) volume ray caster for in situ
 * visualization of simulation fields.
 *
 * The operations follow Matthes et al., "In situ, steerable, hardware-
 * independent and data-structure agnostic visualization with ISAAC"
 * (arXiv:1611.09048):
 *   - sources: scalar or vector fields (feature dimension 1..4) assigned to
 *     every regularly spaced position of the local volume, read in place
 *     through an accessor that handles alignment, pitch and axis order, with
 *     optional guard (ghost) cells and a persistent flag (Sec. 3.1, 3.2 and
 *     the listing "Definition of a source in ISAAC");
 *   - functor chains "f | g | ..." of add, mul, length, sum, pow applied to a
 *     date right after it is read (Sec. 3.3, Tab. "functors");
 *   - free transfer functions, clipping planes and data interpolation
 *     (Sec. 3, feature list);
 *   - one render call that takes control and returns an image (Sec. 3.2).
 *
 * Conventions shared by every call
 *   Coordinates: index space of the local volume.  Voxel (x,y,z) occupies
 *     [x,x+1]x[y,y+1]x[z,z+1]; its value sits at the cell centre; the local
 *     box is [0,Nx]x[0,Ny]x[0,Nz].
 *   Pointers: "device" pointers are HIP device addresses on the context's
 *     device; "host" pointers are ordinary process memory.  Device images
 *     are accessed a pixel at a time: RGBA32F images must be 16-byte
 *     aligned, sample counts, depths and RGBA8 images 4-byte aligned
 *     (ISAAC_ERR_INVALID_ARGUMENT otherwise); source components must be
 *     aligned to their element size.
 *   Ownership: the library never writes to source memory and never frees
 *     memory it did not allocate.  Strings and arrays passed in are copied
 *     before the call returns unless stated otherwise.
 *   Errors: every call returns ISAAC_OK (0) or a negative isaac_status and
 *     never throws or aborts.  A failing set_* call changes nothing.  A
 *     render validates every job before launching any.  A device fault is
 *     reported as ISAAC_ERR_DEVICE, which is sticky: destroy the context.
 *     isaac_last_error() holds a message for the last failure.
 *   Threads: a context is used by one host thread at a time.
 */
#ifndef ISAAC_MI355X_H
#define ISAAC_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISAAC_MAX_SOURCES 8      /* sources per volume */
#define ISAAC_MAX_FUNCTORS 8     /* functors per chain */
#define ISAAC_MAX_CLIP 8         /* clipping planes per render */
#define ISAAC_TF_ENTRIES 256     /* transfer table resolution */
#define ISAAC_MAX_BATCH 256      /* jobs per isaac_render call */

typedef int32_t isaac_status;
enum {
    ISAAC_OK = 0,
    ISAAC_ERR_INVALID_ARGUMENT = -1,
    ISAAC_ERR_BAD_FUNCTOR = -2,      /* functor chain does not parse or has the wrong arity */
    ISAAC_ERR_BAD_TRANSFER = -3,     /* transfer-function points invalid */
    ISAAC_ERR_OUT_OF_MEMORY = -4,
    ISAAC_ERR_BUSY = -5,             /* serving: no slot or memory free right now */
    ISAAC_ERR_NOT_FOUND = -6,        /* unknown volume, handle or ticket */
    ISAAC_ERR_DEVICE = -7            /* HIP error; sticky */
};

typedef enum { ISAAC_F32 = 0, ISAAC_F16 = 1, ISAAC_BF16 = 2 } isaac_dtype;
enum { ISAAC_PERSPECTIVE = 0, ISAAC_ORTHOGRAPHIC = 1 };
enum { ISAAC_NEAREST = 0, ISAAC_TRILINEAR = 1 };
enum { ISAAC_VOLUME = 0, ISAAC_ISO = 1 };     /* render modes */

/* isaac_render flags */
#define ISAAC_ASYNC 1u       /* enqueue on the context stream and return without waiting */
#define ISAAC_TIMING 2u      /* bracket the ray-casting kernel (single-job launches; the whole batched
                                launch otherwise) with HIP events (isaac_timing) */
#define ISAAC_NO_GRAPH 4u    /* batched renders: launch directly instead of replaying a hipGraph */
#define ISAAC_DIRECT 8u      /* read and transform the sources inside the ray loop (no derived volume) */
#define ISAAC_DERIVE 16u     /* use a derived volume whenever the sources allow it (no cost estimate) */

typedef struct isaac_context isaac_context;   /* opaque */

/* isaac_init_desc.flags */
#define ISAAC_INIT_NULL_STREAM 1u   /* with stream == NULL: enqueue on the null stream (HIP's default stream,
                                       which is also PyTorch's default stream), so the context's work is
                                       ordered with work the caller issues there and events the caller records
                                       there bracket it; without this flag a NULL stream asks for a stream of
                                       the context's own, unordered with the caller's */

typedef struct {
    int device;                  /* HIP device ordinal */
    void* stream;                /* hipStream_t to enqueue on (borrowed, never destroyed); NULL: see flags */
    size_t mem_budget_bytes;     /* serving: device bytes for library-owned output images, allocated as one
                                    block at the first isaac_submit*; 0: 1 GiB */
    int max_inflight;            /* serving: outstanding submitted requests; 0: 64 */
    int max_volumes;             /* volume ids 0..max_volumes-1; 0: 256 */
    unsigned flags;              /* ISAAC_INIT_* bits; other bits: ISAAC_ERR_INVALID_ARGUMENT */
} isaac_init_desc;

/* Create a context on a device.  *out receives the context, or NULL on error
 * (use isaac_init_error() for the message then). */
isaac_status isaac_init(const isaac_init_desc* desc, isaac_context** out);

/* Wait for queued work and release everything the library allocated. */
void isaac_destroy(isaac_context* ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* isaac_last_error(const isaac_context* ctx);

/* Message of the last failed isaac_init in this process. */
const char* isaac_init_error(void);

/*
 * Source descriptor (the source concept: feature dimension, guard and
 * persistence flags, name, update callback and accessor; Sec. 3.2).
 *
 * The accessor is a device address per component of interior voxel (0,0,0)
 * and a signed byte stride per axis, so interleaved (AoS) or separate (SoA)
 * components, padded rows, any axis order and reversed axes are all read in
 * place.  Voxel (x,y,z) component c is at comp[c] + x*stride[0] +
 * y*stride[1] + z*stride[2] for x in [-guard, Nx-1+guard] and likewise in y, z.
 * Limits (ISAAC_ERR_INVALID_ARGUMENT otherwise, checked by isaac_set_sources):
 * the kernels address a source with 32-bit byte offsets, so per axis
 * |stride| * (N + 2*g) must stay below 2 GiB, g = min(guard, 1), and so must
 * the byte range the reachable voxels span (all components); strides and
 * component addresses must be multiples of the element size.  A zero stride
 * repeats the field along that axis.  A non-persistent source's packed copy
 * must also stay below 2 GiB.
 */
typedef struct {
    const char* name;                 /* copied; may be NULL */
    int f_dim;                        /* feature dimension, 1..4 */
    isaac_dtype dtype;                /* storage type; arithmetic is FP32 */
    const void* comp[4];              /* device; BORROWED, never written */
    int64_t stride[3];                /* bytes along x, y, z */
    int guard;                        /* guard layers present in memory (0: border clamped under interpolation) */
    int persistent;                   /* 0: the library copies the field after update() into its own buffer */
    const char* functor_chain;        /* e.g. "mul(2,3,4) | add(1) | length"; NULL or "": identity */
    float weight;                     /* in [0,1]: scales the source's opacity when sources are combined */
    int enabled;                      /* 0: never read */
    void (*update)(void* user, int enabled, void* pointer);   /* called before each render; may be NULL */
    void* user;                       /* first argument of update */
} isaac_source_desc;

/* Define (or redefine) volume `volume_id`: its size in cells and its sources.
 * Chains are parsed here (ISAAC_ERR_BAD_FUNCTOR on error).  Every source
 * keeps its current transfer function if the new source count covers it,
 * otherwise it starts with an opacity-0 table until isaac_set_transfer.
 * Must not be called while renders of this volume are in flight. */
isaac_status isaac_set_sources(isaac_context* ctx, int volume_id, const int32_t dims[3],
                               const isaac_source_desc* src, int n_src);

/* Piecewise-linear RGBA transfer function over the classification domain
 * [0,1]: x strictly increasing from 0 to 1, every value in [0,1].  It is
 * tabulated at 256 points j/255 and looked up with linear interpolation; a
 * value outside [0,1] is clamped, NaN maps to 0. */
typedef struct { double x; double rgba[4]; } isaac_tf_point;

/* Bake and upload a table, make it the current table of (volume, source) and
 * return its handle (>= 0) in *out_handle (may be NULL).  Handles stay valid
 * until isaac_release_transfer. */
isaac_status isaac_set_transfer(isaac_context* ctx, int volume_id, int source,
                                const isaac_tf_point* pts, int n_pts, int32_t* out_handle);

/* Give a table back; its slot is reused once no queued render refers to it.
 * Releasing a source's current table leaves it current until replaced. */
isaac_status isaac_release_transfer(isaac_context* ctx, int32_t handle);

typedef struct { double n[3]; double d; } isaac_clip_plane;   /* keep points with n.x + d >= 0 */

typedef struct {
    int volume_id;
    int width, height;                /* image size in pixels, >= 1 */
    int projection;                   /* ISAAC_PERSPECTIVE or ISAAC_ORTHOGRAPHIC */
    double eye[3], center[3], up[3];  /* camera, index-space units; right = forward x up; eye != center;
                                         up not within 1e-6 rad of the view direction */
    double fovy_deg;                  /* perspective: vertical field of view, (0,180) */
    double ortho_height;              /* orthographic: image height in voxels, > 0 */
    double step;                      /* sample spacing along the ray in voxels, > 0 */
    int interpolation;                /* ISAAC_NEAREST or ISAAC_TRILINEAR */
    int n_clip;                       /* <= ISAAC_MAX_CLIP */
    const isaac_clip_plane* clip;     /* host; copied */
    const int32_t* tf_handles;        /* host, one per source; NULL: the current tables */
    const float* weights;             /* host, one per source; NULL: descriptor weights */
    const int32_t* enabled;           /* host, one per source; NULL: descriptor flags */
    float ert_threshold;              /* stop a ray once opacity >= this; 0: 0.999; > 1: never */
    float* out_rgba;                  /* device, CALLER-OWNED, height*width*4 floats, premultiplied, row 0 = top */
    int32_t* out_samples;             /* device or NULL: per-pixel count of composited samples */
    void* update_pointer;             /* passed as `pointer` to every source's update() */
    /* Brick of a larger volume (sort-last rendering, Sec. 3.1): when
     * brick_origin is not NULL the camera and clip planes are in the global
     * index space [0, global_dims], the step grid is anchored at the entry into
     * the global box, and this volume (voxel (0,0,0) at brick_origin) renders
     * only the scan points inside its own box.  Neighbouring bricks split every
     * ray's scan points without overlap; isaac_composite combines the partial
     * images.  Use ert_threshold > 1 for bricks: termination needs the opacity
     * in front, which a brick does not know. */
    const int32_t* brick_origin;      /* host, 3 ints, or NULL */
    const int32_t* global_dims;       /* host, 3 ints (required with brick_origin) */
    float* out_depth;                 /* device or NULL: per pixel, ray parameter of the first scan point
                                         (+inf where there is none), the compositing order */
    /* Render mode.  ISAAC_VOLUME: emission-absorption compositing of every
     * source (Sec. 3.2).  ISAAC_ISO: iso-surfaces (a listed feature of Sec. 3):
     * the same scan points; the surface is the first place where a source's
     * interpolated, functor-transformed value crosses that source's iso
     * value between two consecutive scan points, placed by linear
     * interpolation between them; the pixel is opaque, coloured by the
     * source's transfer function at the iso value times
     * 0.3 + 0.7 |cos| of the angle between the ray and the central-difference
     * gradient (half a voxel each side).  Weights and ert_threshold are
     * unused; out_samples counts scan points up to and including the one
     * after the crossing.  Not combinable with brick_origin. */
    int32_t mode;                     /* ISAAC_VOLUME (0) or ISAAC_ISO */
    const float* iso_values;          /* host, one per source (ISAAC_ISO); NaN: the source draws no surface
                                         and is not read; NULL: no source draws one */
} isaac_render_desc;

/* Ray-cast jobs (all validated before any launch).  One job is one kernel
 * launch over its image; several jobs form one persistent launch over a
 * shared tile queue, replayed as a hipGraph unless ISAAC_NO_GRAPH.  Without
 * ISAAC_ASYNC the call returns after the images are complete.
 * Derived volume: when the call's expected scan points on a volume (8 voxel
 * visits each under trilinear interpolation) exceed 4 per voxel, or with
 * ISAAC_DERIVE, and at most 4 of its sources are active, the call first
 * evaluates every active source's functor chain once per voxel (guards
 * included) into a library-owned FP32 buffer of 4 bytes per voxel and source
 * (plus up to two padding layers per axis), kept per volume until it is
 * redefined, and the ray loop reads that buffer.
 * The image is the same bit for bit.  ISAAC_DIRECT never derives.  Serving
 * calls (isaac_submit*) never derive. */
isaac_status isaac_render(isaac_context* ctx, const isaac_render_desc* jobs, int n_jobs, unsigned flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the render of
 * isaac_render, with the same images bit for bit, that calls no hipMalloc,
 * hipFree or other allocating routine.
 *   - The set-up pass writes its ray records (40 bytes per pixel of each job's
 *     screen rectangle, the projected box) into a static device array of
 *     ISAAC_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 *     on until the process ends.  A call whose jobs' rectangles together need
 *     more is refused with ISAAC_ERR_INVALID_ARGUMENT before anything runs (at
 *     most 838860 rectangle pixels: e.g. any 1024x768 job, or a 1920x1080 job
 *     whose volume covers up to 40 % of the screen).
 *   - No derived volume is built: a frozen volume's derived values are read
 *     (isaac_freeze_volume), other volumes are read in place, as with
 *     ISAAC_DIRECT.  Non-persistent sources are copied into the buffers
 *     isaac_set_sources allocated.
 *   - Batches are launched directly (no hipGraph); no pooled schedule.
 *   - flags: ISAAC_ASYNC, ISAAC_NO_GRAPH, ISAAC_DIRECT; any other bit
 *     (ISAAC_TIMING, ISAAC_DERIVE) is ISAAC_ERR_INVALID_ARGUMENT.
 * Every call on a device shares that device's array, whose contents the next
 * call overwrites: calls that overlap on one device (on other streams or from
 * other contexts) race and must be ordered by the caller; calls on one
 * context's stream are ordered already. */
#define ISAAC_NOALLOC_SCRATCH_BYTES (32u << 20)
isaac_status isaac_render_noalloc(isaac_context* ctx, const isaac_render_desc* jobs, int n_jobs, unsigned flags);

/* Sort-last compositing (Sec. 3.1, Fig. "whole concept"): per pixel, order the
 * n_layers partial images by their depth images (out_depth of the brick
 * renders) and combine them front to back:
 * (C, A) o (C', A') = (C + (1-A) C', A + (1-A) A'), equal depths in layer
 * order.  A depth of +inf marks a pixel the layer does not cover (a brick
 * render writes +inf and colour (0,0,0,0) where it keeps no scan point): the
 * layer's colour there is not read; a pixel no layer covers is (0,0,0,0).
 * rgba and depth are host arrays of n_layers device pointers (1..16); out is
 * device RGBA32F.  Runs on the context stream; without ISAAC_ASYNC it waits
 * for the result. */
isaac_status isaac_composite(isaac_context* ctx, const float* const* rgba, const float* const* depth, int n_layers,
                             int width, int height, float* out, unsigned flags);

/* Freeze a volume whose sources will not change until it is redefined (a
 * resident data set explored by many renders or served requests): every
 * source's functor chain is evaluated once per voxel now (guards included),
 * into the library-owned derived volume of 4 bytes per voxel and source, and
 * every later render or served request of the volume, whatever its clip
 * planes and enabled sources, reads those values instead of the sources (with
 * three sources, whose values are stored for the three-source loop, an
 * iso-surface job or one with fewer active sources reads the sources).
 * Images are the same bit for bit.  The sources must be persistent and at
 * most 4; their update callbacks are called once here and still before each
 * render.  The caller must not change the sources' memory while the volume is
 * frozen; isaac_set_sources (redefinition) thaws it.  A volume whose sources
 * are read directly anyway (plain packed FP32 scalars) stays as it is.
 * Synchronous: returns when the derived values are complete. */
isaac_status isaac_freeze_volume(isaac_context* ctx, int volume_id);

/* Frame encode (the step after compositing, where the root rank compresses
 * the image before sending it, Sec. 3.6): each pixel of a premultiplied
 * RGBA32F image (device, width*height*4 floats) is quantized to 8 bits per
 * channel into out (device, width*height*4 bytes, row 0 on top):
 *   background == NULL: (q(C_r), q(C_g), q(C_b), q(A)), still premultiplied;
 *   background = host rgb in [0,1]: (q(C_c + (1-A) bg_c), ..., 255), the
 *     image over an opaque background;
 * with q(v) = floor(clamp(v, 0, 1) * 255 + 1/2) and NaN -> 0, every step a
 * separately rounded FP32 operation.  Runs on the context stream; without
 * ISAAC_ASYNC it waits for the result. */
isaac_status isaac_encode_rgba8(isaac_context* ctx, const float* rgba, int width, int height,
                                const float* background, unsigned char* out, unsigned flags);

/* JPEG compression of an RGBA8 frame, the form in which the root rank sends
 * the composited image to the server (Sec. 3.6).  The paper leaves the
 * encoder open; this one writes baseline sequential JPEG (JFIF 1.01):
 *  - colour: Y, Cb, Cr from R, G, B (alpha ignored) with the JFIF weights in
 *    16-bit fixed point, each rounded half up by a shift; no subsampling;
 *  - 8x8 blocks in raster order, the frame extended by repeating its last
 *    column and row; samples minus 128;
 *  - forward DCT with the cosine matrix rounded to 12 fractional bits, the
 *    row pass keeping 2 fractional bits, both passes rounded half up by shifts;
 *  - the example tables of the JPEG standard (Annex K) scaled by quality
 *    (1..100; 5000/q percent below 50, else 200 - 2q), quotients rounded half
 *    away from zero;
 *  - four Huffman tables (DC and AC, luma and chroma) built for this frame
 *    from its symbol counts by the procedure of Annex K.2 (ties to the larger
 *    symbol value, lengths limited to 16 bits), canonical codes;
 *  - last byte padded with 1 bits, 0x00 after every 0xFF data byte.
 * rgba8: device, width*height*4 bytes, row 0 on top; width and height in
 * 1..65535.  out: host, capacity bytes; *out_size receives the stream's size,
 * also when capacity is too small (then ISAAC_ERR_INVALID_ARGUMENT and out is
 * not written).  The stream is a fixed function of (pixels, quality).  Runs on
 * the context stream (ordered after earlier work there) and returns when the
 * stream is in out.  Device scratch, sized for the largest stream the frame
 * can give (about 42 bytes per pixel), is kept by the context between calls
 * and grows with the frame size; device errors are ISAAC_ERR_DEVICE. */
isaac_status isaac_encode_jpeg(isaac_context* ctx, const unsigned char* rgba8, int width, int height, int quality,
                               unsigned char* out, size_t capacity, size_t* out_size);

/* Sum and count of the kernel durations of ISAAC_TIMING renders since the
 * last call (waits for them), then resets. */
isaac_status isaac_timing(isaac_context* ctx, double* total_ms, int* count);

/* Ray-tile shape and scan-point schedule for jobs of one image-size class
 * (the autotuner's output).  size_class = ceil(log2(max(width,height)))
 * clamped to [0,15].
 *   lanes_per_ray in {1,2,4,8,16,32,64}: lanes sharing one ray, each taking
 *     every lanes_per_ray-th scan point (more parallelism where few rays meet
 *     the volume); a 64-lane wave holds 64/lanes_per_ray rays;
 *   wave_w, a power of two in [1, 64/lanes_per_ray]: a wave's rays form a
 *     wave_w x (64/lanes_per_ray/wave_w) pixel block;
 *   waves_x in {1,2,4}: the 4 waves of a workgroup are waves_x x 4/waves_x;
 *   unroll in {1,2} (one lane per ray only): scan points whose source reads
 *     are issued together;
 *   min_waves in {0,4}: 4 selects the kernel variant compiled to keep at
 *     least 4 waves resident per SIMD (not with lanes_per_ray 2, 32, 64 or
 *     unroll 2);
 *   pooled in {0,1} (lanes_per_ray 2..16): a render call's single-job
 *     launches first set up every pixel's ray and compact the rays that keep
 *     scan points into a list, then resident waves hand those rays to lane
 *     groups as groups free up (no lanes idle on short or missing rays).
 *     Only isaac_render uses it (a library-owned list of 40 bytes per pixel,
 *     kept in the context); serving and batched launches use the tiles.
 * A batch runs one launch per distinct schedule, so each job is rendered as
 * it would be alone.
 * Defaults: (8, 2, 1, 1, 0, 0).  Settings with one lane per ray give the same
 * image bit for bit; more lanes composite each row of scan points by a scan,
 * which changes only FP32 rounding; a given setting always reproduces its
 * image bit for bit. */
isaac_status isaac_set_tile_shape(isaac_context* ctx, int size_class, int wave_w, int waves_x, int unroll,
                                  int lanes_per_ray, int min_waves, int pooled);
isaac_status isaac_get_tile_shape(isaac_context* ctx, int size_class, int* wave_w, int* waves_x, int* unroll,
                                  int* lanes_per_ray, int* min_waves, int* pooled);

/* ---- serving: library-owned output images admitted against mem_budget ---- */

/* Enqueue one render into a library-owned image (job->out_rgba and
 * job->out_samples are ignored).  Images are carved from the memory budget
 * (one device block, allocated at the first submission; images in 256-byte
 * granules, first fit), so later submissions allocate no device memory.
 * Returns ISAAC_ERR_BUSY when max_inflight requests are outstanding or the
 * image does not fit a free run of the budget. */
isaac_status isaac_submit(isaac_context* ctx, const isaac_render_desc* job, uint64_t* out_ticket);

/* Several requests as one batched launch; tickets[i] receives job i's ticket.
 * All or nothing: ISAAC_ERR_BUSY if any of them would not be admitted. */
isaac_status isaac_submit_batch(isaac_context* ctx, const isaac_render_desc* jobs, int n_jobs,
                                uint64_t* tickets);

/* *done = 1 once the image is complete; *out_rgba then points at it (device,
 * owned by the library until isaac_release). */
isaac_status isaac_poll(isaac_context* ctx, uint64_t ticket, int* done, const float** out_rgba);

/* Copy a ticket's image (waiting for it) into host memory of height*width*4
 * floats. */
isaac_status isaac_read_image(isaac_context* ctx, uint64_t ticket, float* host_rgba);

/* Encode a ticket's image as isaac_encode_rgba8 does (waiting for it) and copy
 * the height*width*4 bytes into host memory: a quarter of the RGBA32F copy.
 * background: host rgb in [0,1] or NULL. */
isaac_status isaac_read_image_rgba8(isaac_context* ctx, uint64_t ticket, const float* background,
                                    unsigned char* host_rgba8);

/* Encode a ticket's image to RGBA8 as isaac_read_image_rgba8 does, then to
 * JPEG as isaac_encode_jpeg does (waiting for both): what the root rank sends
 * to the server (Sec. 3.6). */
isaac_status isaac_read_image_jpeg(isaac_context* ctx, uint64_t ticket, const float* background, int quality,
                                   unsigned char* out, size_t capacity, size_t* out_size);

/* Return the image memory of a completed (or not yet complete: waits) ticket. */
isaac_status isaac_release(isaac_context* ctx, uint64_t ticket);

/* Bytes of the serving memory budget in use / in total. */
isaac_status isaac_serving_usage(isaac_context* ctx, size_t* used, size_t* budget, int* inflight);

/* ---- host-only helpers (no device needed) ---- */

/* Parse a functor chain for an f_dim-component source: *out_dim receives the
 * dimension of the chain's result, *out_ops the number of functors after
 * host-side simplification.  Message in err on ISAAC_ERR_BAD_FUNCTOR. */
isaac_status isaac_check_functor_chain(const char* chain, int f_dim, int* out_dim, int* out_ops,
                                       char* err, int errlen);

/* Library version string. */
const char* isaac_version(void);

#ifdef __cplusplus
}
#endif
#endif
