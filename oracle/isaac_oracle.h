/*
 * FP64 single-threaded CPU oracle of the ISAAC volume ray caster.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; the
 * library never links, loads or calls it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (Matthes et al., "In situ, steerable, hardware-independent
 * and data-structure agnostic visualization with ISAAC"):
 *   - one ray per pixel through the local volume (Sec. 3.1, Fig. "whole concept");
 *   - at every scan point, for every enabled source: read the date through the
 *     source's accessor at integer indices, apply the source's functor chain,
 *     interpolate (trilinear) or take the nearest cell, classify through the
 *     transfer function, and combine all sources into one colour and opacity
 *     (Sec. 3.2, the paragraph after Fig. "pap"; Sec. 3.3, Tab. "functors");
 *   - classical front-to-back compositing (Sec. 3.2);
 *   - guard cells remove the border check under interpolation (Sec. 3.2);
 *   - disabled sources are never read (Sec. 3.2, the 2^n render functions);
 *   - clipping planes and free transfer functions (Sec. 3, feature list).
 * Where the paper is silent the readings are the ones listed in the design
 * notes of this repository (cell-centred samples, half-step grid anchored at
 * the box entry, premultiplied weighted mixing, early termination at theta).
 */
#ifndef ISAAC_ORACLE_H
#define ISAAC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_F32 = 0, ORACLE_F16 = 1, ORACLE_BF16 = 2 };

typedef struct {
    int f_dim;                        /* 1..4 */
    int dtype;                        /* ORACLE_F32 / F16 / BF16 */
    const unsigned char* comp[4];     /* host address of component c of interior voxel (0,0,0) */
    int64_t stride[3];                /* signed byte strides along x, y, z */
    int guard;                        /* >= 1: a guard layer exists, no border clamp */
    const char* chain;                /* functor chain text; NULL or "" = identity */
    double weight;
    int enabled;                      /* 0: never read */
    int n_tf;                         /* number of transfer-function control points */
    const double* tf;                 /* n_tf * 5 doubles: x r g b a */
    double iso;                       /* iso-surface mode: the source's iso value (NaN: no surface) */
} oracle_source;

typedef struct {
    int dims[3];                      /* local volume in cells, x y z */
    int n_src;
    const oracle_source* src;
    int orthographic;
    double eye[3], center[3], up[3];
    double fovy_deg, ortho_height;
    int width, height;
    double step;                      /* sample spacing along the ray, voxels */
    int interpolation;                /* 0 nearest, 1 trilinear */
    int n_clip;
    const double* clip;               /* n_clip * 4: nx ny nz d, keep n.x + d >= 0 */
    double ert_threshold;             /* stop once accumulated opacity >= this (> 1: never) */
    int mode;                         /* 0 volume rendering, 1 iso-surface rendering */
    double iso_margin;                /* iso mode: relative arithmetic error of a value (the decision margin of
                                         the iso comparison adds the value's change over +-delta per axis) */
    double delta;                     /* decision margin for the flip allowance (voxels) */
    double ert_margin;                /* opacity margin for the flip allowance at the threshold */
} oracle_scene;

typedef struct {
    double rgba[4];                   /* premultiplied colour and opacity */
    int64_t samples;                  /* scan points composited */
    double allowance;                 /* per-channel bound on what a flipped decision can change */
    int32_t flags;                    /* decisions taken within the margin */
    int32_t kinds;                    /* ORACLE_FLAG_* bits of those decisions */
    int32_t count_slack;              /* how far the sample count may move (clip plane and box exit) */
    int32_t pad;
} oracle_pixel;

enum { ORACLE_FLAG_NEAREST = 1, ORACLE_FLAG_CLIP = 2, ORACLE_FLAG_EXIT = 4, ORACLE_FLAG_ERT = 8, ORACLE_FLAG_ISO = 16 };

/* Render pixels [first, first+count) of the row-major image (row 0 at the top).
 * Returns 0, or -1 with a message in err. */
int oracle_render_range(const oracle_scene* sc, int64_t first, int64_t count,
                        oracle_pixel* out, char* err, int errlen);

/* Render the listed pixels: px holds n (column, row) pairs. */
int oracle_render_list(const oracle_scene* sc, const int32_t* px, int64_t n,
                       oracle_pixel* out, char* err, int errlen);

/* Apply a functor chain to one f_dim-component date; *out is the value used for
 * classification (component 0 of the result), *out_dim the result dimension. */
int oracle_chain_eval(const char* chain, int f_dim, const double* in, double* out,
                      int* out_dim, char* err, int errlen);

/* The 256-entry transfer table T[j] = PL(j/255), 256 * 4 doubles. */
int oracle_tf_table(int n_tf, const double* tf, double* table, char* err, int errlen);

/* Ray of pixel (i, j): origin, unit direction and the box interval [t0, t1]
 * (t0 >= 0); returns 1 if the ray meets the box, 0 otherwise. */
/* Frame encode (the image is compressed before it is sent, Sec. 3.6): each
 * premultiplied RGBA pixel, optionally over an opaque rgb background, is
 * quantized to 8 bits, q(v) = floor(clamp(v,0,1)*255 + 1/2), NaN -> 0.  The
 * quantization is an integer decision, taken here in FP32 with every
 * operation rounded separately (the precision of the library's output). */
void oracle_encode_rgba8(const float* rgba, int64_t n_pixels, const float* background, unsigned char* out);

int oracle_ray(const oracle_scene* sc, int i, int j, double o[3], double d[3],
               double* t0, double* t1);

#ifdef __cplusplus
}
#endif
#endif
