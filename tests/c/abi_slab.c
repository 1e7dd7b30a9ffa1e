/* A C99 caller of the library: no Python, no torch.  Renders a constant slab
 * (every voxel 0.5, one guard layer) seen orthographically along +x with a
 * constant transfer function, and checks every pixel against the closed form
 * of front-to-back compositing of n equal samples of opacity a and colour c:
 * A = 1 - (1 - a)^n, C = c A (premultiplied).  A ray through the whole box
 * takes 16 / 0.5 = 32 scan points.  Exit status 0 when all pixels agree.
 * Test infrastructure (built and run by tests/test_c_abi.py). */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "isaac_mi355x.h"

#define N 16
#define W 24
#define H 24

static int fail(const char* what, const char* msg) {
    fprintf(stderr, "abi_slab: %s: %s\n", what, msg);
    return 1;
}

int main(void) {
    const size_t ext = N + 2, nvox = ext * ext * ext;
    float* host = (float*)malloc(nvox * sizeof(float));
    for (size_t i = 0; i < nvox; ++i) host[i] = 0.5f;
    float *vol = NULL, *rgba = NULL;
    int32_t* samples = NULL;
    if (hipMalloc((void**)&vol, nvox * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&rgba, (size_t)W * H * 4 * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&samples, (size_t)W * H * sizeof(int32_t)) != hipSuccess)
        return fail("hipMalloc", "failed");
    if (hipMemcpy(vol, host, nvox * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return fail("hipMemcpy", "failed");

    isaac_init_desc idesc = {0};
    isaac_context* ctx = NULL;
    if (isaac_init(&idesc, &ctx) != ISAAC_OK) return fail("isaac_init", isaac_init_error());

    isaac_source_desc src = {0};
    src.name = "slab";
    src.f_dim = 1;
    src.dtype = ISAAC_F32;
    src.comp[0] = vol + 1 + ext + ext * ext;             /* interior voxel (0,0,0) */
    src.stride[0] = sizeof(float);
    src.stride[1] = (int64_t)(ext * sizeof(float));
    src.stride[2] = (int64_t)(ext * ext * sizeof(float));
    src.guard = 1;
    src.persistent = 1;
    src.weight = 1.0f;
    src.enabled = 1;
    const int32_t dims[3] = {N, N, N};
    if (isaac_set_sources(ctx, 0, dims, &src, 1) != ISAAC_OK) return fail("isaac_set_sources", isaac_last_error(ctx));
    const double c[3] = {0.2, 0.4, 0.6}, a = 0.05;
    const isaac_tf_point tf[2] = {{0.0, {c[0], c[1], c[2], a}}, {1.0, {c[0], c[1], c[2], a}}};
    if (isaac_set_transfer(ctx, 0, 0, tf, 2, NULL) != ISAAC_OK) return fail("isaac_set_transfer", isaac_last_error(ctx));

    isaac_render_desc rd = {0};
    rd.volume_id = 0;
    rd.width = W;
    rd.height = H;
    rd.projection = ISAAC_ORTHOGRAPHIC;
    rd.eye[0] = -20.0, rd.eye[1] = 8.0, rd.eye[2] = 8.0;
    rd.center[0] = 8.0, rd.center[1] = 8.0, rd.center[2] = 8.0;
    rd.up[2] = 1.0;
    rd.ortho_height = 20.0;
    rd.step = 0.5;
    rd.interpolation = ISAAC_TRILINEAR;
    rd.ert_threshold = 2.0f;                             /* no early termination */
    rd.out_rgba = rgba;
    rd.out_samples = samples;
    if (isaac_render(ctx, &rd, 1, 0) != ISAAC_OK) return fail("isaac_render", isaac_last_error(ctx));

    float* img = (float*)malloc((size_t)W * H * 4 * sizeof(float));
    int32_t* cnt = (int32_t*)malloc((size_t)W * H * sizeof(int32_t));
    if (hipMemcpy(img, rgba, (size_t)W * H * 4 * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(cnt, samples, (size_t)W * H * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy", "failed");
    int hit = 0, full = 0, bad = 0;
    double worst = 0.0;
    for (int p = 0; p < W * H; ++p) {
        const int n = cnt[p];
        const double A = n > 0 ? 1.0 - pow(1.0 - (double)(float)a, n) : 0.0;
        double e = fabs(img[4 * p + 3] - A);
        for (int k = 0; k < 3; ++k) e = fmax(e, fabs(img[4 * p + k] - (double)(float)c[k] * A));
        worst = fmax(worst, e);
        if (e > 1e-5 || n < 0 || n > 32) ++bad;
        hit += n > 0;
        full += n == 32;
    }
    printf("abi_slab: %d of %d pixels hit the slab, %d with 32 scan points; worst error %.3g; %d bad\n", hit, W * H,
           full, worst, bad);
    isaac_destroy(ctx);
    hipFree(vol);
    hipFree(rgba);
    hipFree(samples);
    free(host);
    free(img);
    free(cnt);
    return (bad == 0 && full > 0 && hit < W * H) ? 0 : 2;
}
