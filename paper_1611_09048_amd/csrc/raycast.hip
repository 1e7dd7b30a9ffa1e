// Volume ray casting kernels for gfx950 (MI355X).
//
// One ray per lane; a 64-lane wave covers a wave_w x (64/wave_w) pixel
// block and a 256-thread workgroup a 2-D arrangement of four such blocks.
// For every pixel the kernel builds the ray in FP64, intersects it with the
// local box and the clipping planes (the kept scan points along a ray form
// one interval of the sample index k), then marches in FP32: at each scan
// point every active source is read at integer indices through its strided
// accessor, passed through its functor chain, interpolated (trilinear) or
// taken from the nearest cell, classified with its transfer table, weighted
// and mixed into one colour and opacity, and composited front to back until
// the opacity reaches the termination threshold.  This is the per-scan-point
// source loop of ISAAC (Matthes et al., Sec. 3.2, Fig. "pap" and the
// paragraph after it; functors Sec. 3.3, Tab. "functors").
//
// Source reads use raw buffer loads: a read outside the range the host
// derived from the declared extents returns 0 instead of touching memory.
// Transfer tables (256 x RGBA32F per source) live in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "isaac_internal.h"

namespace isaac {

namespace {

constexpr int kRsrcFlags = 0x00020000;   // raw buffer, 32-bit data format (gfx9 family)

// Source descriptors are wave-uniform by construction; readfirstlane keeps
// the buffer resource in SGPRs whatever the compiler could prove.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(uint64_t base, uint32_t n) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const uint64_t b = ((uint64_t)hi << 32) | lo;
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(b), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(n), kRsrcFlags);
}

__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ __forceinline__ float ld_scalar(__amdgpu_buffer_rsrc_t r, int off, int dtype) {
    if (dtype == DT_F32) return ld_f32(r, off);
    unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    if (dtype == DT_F16) return (float)__builtin_bit_cast(_Float16, h);
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// N voxels of one source (N = 1 nearest, 8 trilinear corners); off[i] is the
// byte offset of voxel i relative to voxel (0,0,0).  One uniform branch per
// call selects the load form, and all N loads are issued before any is used.
template <int N>
__device__ __forceinline__ void fetch(const DevSource& S, const int (&off)[N], float (&v)[N][4]) {
    const int f_dim = S.f_dim;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i][0] = v[i][1] = v[i][2] = v[i][3] = 0.f;
    if (S.packed && S.dtype == DT_F32) {
        // adjacent FP32 components: consecutive dword loads merge into x2/x3/x4 loads
        const __amdgpu_buffer_rsrc_t r = make_rsrc(S.base[0], S.num_records[0]);
        const int o = S.comp_off[0];
        if (f_dim == 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) v[i][0] = ld_f32(r, off[i] + o);
        } else if (f_dim == 3) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v[i][0] = ld_f32(r, off[i] + o);
                v[i][1] = ld_f32(r, off[i] + o + 4);
                v[i][2] = ld_f32(r, off[i] + o + 8);
            }
        } else if (f_dim == 2) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v[i][0] = ld_f32(r, off[i] + o);
                v[i][1] = ld_f32(r, off[i] + o + 4);
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v[i][0] = ld_f32(r, off[i] + o);
                v[i][1] = ld_f32(r, off[i] + o + 4);
                v[i][2] = ld_f32(r, off[i] + o + 8);
                v[i][3] = ld_f32(r, off[i] + o + 12);
            }
        }
        return;
    }
    const int dtype = S.dtype;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c < f_dim) {
            const int k = S.packed ? 0 : c;
            const __amdgpu_buffer_rsrc_t r = make_rsrc(S.base[k], S.num_records[k]);
            const int o = S.comp_off[c];
#pragma unroll
            for (int i = 0; i < N; ++i) v[i][c] = ld_scalar(r, off[i] + o, dtype);
        }
    }
}

// pow for FP32 with IEEE special cases: exp2(y log2|x|), a negative base
// needs an integer exponent (odd exponents keep the sign), else NaN.
__device__ __forceinline__ float pow_f32(float x, float y) {
    if (y == 0.f) return 1.f;
    if (x == 1.f) return 1.f;
    float ax = fabsf(x);
    float r;
    if (ax == 0.f) {
        r = (y > 0.f) ? 0.f : __builtin_inff();
    } else {
        r = __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(ax));
    }
    if (x < 0.f) {
        float yi = truncf(y);
        if (yi != y) return __builtin_nanf("");
        float half = 0.5f * yi;
        if (truncf(half) != half) r = -r;   // odd exponent
    }
    return r;
}

// Functor chain over N dates at once: one wave-uniform dispatch per functor,
// N dates of work inside.  D bounds the feature dimension at compile time
// (components D..3 are never touched); res[i] is component 0 of date i's
// result.
template <int N, int D = 4>
__device__ __forceinline__ void run_chain_n(const DevSource& S, float (&v)[N][4], float (&res)[N]) {
    const int n_ops = S.n_ops;
    for (int o = 0; o < n_ops; ++o) {
        const DevOp& op = S.ops[o];
        const int dim = op.dim;
        const float a[4] = {op.arg[0], op.arg[1], op.arg[2], op.arg[3]};
        switch (op.kind) {
        case OP_ADD:
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] + a[c];
            break;
        case OP_MUL:
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] * a[c];
            break;
        case OP_POW:
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = pow_f32(v[i][c], a[c]);
            break;
        case OP_SQRT:
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i)
                        v[i][c] = v[i][c] < 0.f ? __builtin_nanf("") : __builtin_amdgcn_sqrtf(v[i][c]);
            break;
        case OP_SQUARE:
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] * v[i][c];
            break;
        case OP_LENGTH:
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float s = v[i][0] * v[i][0];
                if (D > 1 && dim > 1) s = fmaf(v[i][1], v[i][1], s);
                if (D > 2 && dim > 2) s = fmaf(v[i][2], v[i][2], s);
                if (D > 3 && dim > 3) s = fmaf(v[i][3], v[i][3], s);
                v[i][0] = __builtin_amdgcn_sqrtf(s);
            }
            break;
        case OP_SUM:
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float s = v[i][0];
                if (D > 1 && dim > 1) s = s + v[i][1];
                if (D > 2 && dim > 2) s = s + v[i][2];
                if (D > 3 && dim > 3) s = s + v[i][3];
                v[i][0] = s;
            }
            break;
        default:
            break;
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) res[i] = v[i][0];
}

// The 8 trilinear corners run the bytecode in two groups of 4, which bounds
// the interpreter's live registers (more resident waves).
template <int N, int D = 4>
__device__ __forceinline__ void run_chain(const DevSource& S, float (&v)[N][4], float (&res)[N]) {
    if constexpr (N == 8) {
        float a[4][4], b[4][4], ra[4], rb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a[i][c] = v[i][c];
                b[i][c] = v[i + 4][c];
            }
        run_chain_n<4, D>(S, a, ra);
        run_chain_n<4, D>(S, b, rb);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            res[i] = ra[i];
            res[i + 4] = rb[i];
        }
    } else {
        run_chain_n<N, D>(S, v, res);
    }
}

// Transfer-table lookup in a staged table (kTfLds values): clamp to [0,1]
// (NaN -> 0), 255 intervals, linear.  No contraction: the fraction is that of
// the rounded u in every caller, whatever the surrounding code lets the
// compiler fuse.  u is in [0, 255], so its fraction is exact and equals u - j;
// at u = 255 the lookup lands on the last entry, whose copy makes the slope 0,
// and returns T[255] itself.
__device__ __forceinline__ float4 classify(const float4* __restrict__ table, float x) {
#pragma clang fp contract(off)
    float t = fminf(fmaxf(x, 0.f), 1.f);    // max(NaN, 0) = 0
    float u = 255.f * t;
    int j = (int)u;
    float f = __builtin_amdgcn_fractf(u);
    const float4 a = table[j];              // T[j]
    const float4 b = table[j + 1];          // T[j+1]
    return make_float4(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y), fmaf(f, b.z - a.z, a.z),
                       fmaf(f, b.w - a.w, a.w));
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// FP64 ray setup.  Returns false if the ray misses the box or keeps no scan
// point; otherwise the kept sample indices are [*kb, *ke) and the FP32 ray is
// p(k) = pb + ((k + 1/2) * step) * d32.
struct RaySetup {
    float pb[3];           // global position of the ray at t0
    float d[3];
    int kb, ke;
    float t_first;         // ray parameter of scan point kb
};

// A set-up ray as stored by the setup passes (40 bytes).
struct RayRec {
    float pb[3];
    float d[3];
    int kb, ke;
    float t_first;
    int pixel;
};

// Scan point k in the volume's own index space: the global position minus the
// brick origin (an exact FP32 subtraction of an integer below the position).
__device__ __forceinline__ void point_at(const DevJob& J, const RaySetup& R, float tk, float (&p)[3]) {
    p[0] = fmaf(tk, R.d[0], R.pb[0]) - J.org[0];
    p[1] = fmaf(tk, R.d[1], R.pb[1]) - J.org[1];
    p[2] = fmaf(tk, R.d[2], R.pb[2]) - J.org[2];
}

// Trilinear cell coordinates u = p - 1/2 of scan point k in index space:
// the numbers point_at at (k + 1/2) step gives, minus 1/2, bit for bit, in
// fewer operations.  (k + 1/2) step and k step + step/2 are the same real
// number, rounded once either way; position - org is exact (an integer origin
// below 2^22, a position at most a voxel outside the brick), so subtracting
// org + 1/2 at once rounds the same value as subtracting org, then 1/2.
__device__ __forceinline__ void cell_at(const DevJob& J, const RaySetup& R, int k, float (&u)[3]) {
    const float tk = fmaf((float)k, (float)J.step, J.half_step);
    u[0] = fmaf(tk, R.d[0], R.pb[0]) - J.orgh[0];
    u[1] = fmaf(tk, R.d[1], R.pb[1]) - J.orgh[1];
    u[2] = fmaf(tk, R.d[2], R.pb[2]) - J.orgh[2];
}

__device__ __forceinline__ bool setup_ray(const DevJob& J, int px, int py, RaySetup& R) {
#pragma clang fp contract(off)
    const double x = (2.0 * (px + 0.5) / J.width - 1.0) * J.h * J.aspect;
    const double y = (1.0 - 2.0 * (py + 0.5) / J.height) * J.h;
    double o[3], d[3];
    if (J.ortho) {
        for (int a = 0; a < 3; ++a) {
            o[a] = J.eye[a] + x * J.right[a] + y * J.upp[a];
            d[a] = J.fwd[a];
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            o[a] = J.eye[a];
            d[a] = J.fwd[a] + x * J.right[a] + y * J.upp[a];
        }
        const double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; ++a) d[a] = d[a] / n;
    }
    // slab test against the box [lo_a, hi_a] per axis
    auto slab = [&](const double* blo, const double* bhi, double& lo, double& hi) {
#pragma clang fp contract(off)
        lo = -__builtin_inf();
        hi = __builtin_inf();
        for (int a = 0; a < 3; ++a) {
            if (d[a] == 0.0) {
                if (o[a] < blo[a] || o[a] > bhi[a]) return false;
                continue;
            }
            const double ta = (blo[a] - o[a]) / d[a];
            const double tb = (bhi[a] - o[a]) / d[a];
            const double tn = ta < tb ? ta : tb;
            const double tf = ta < tb ? tb : ta;
            if (tn > lo) lo = tn;
            if (tf < hi) hi = tf;
        }
        return true;
    };
    // the step grid is anchored at the entry into the global box
    const double zero[3] = {0.0, 0.0, 0.0};
    double lo, hi;
    if (!slab(zero, J.gbox_hi, lo, hi)) return false;
    if (lo < 0.0) lo = 0.0;
    if (!(hi > lo)) return false;
    const double t0 = lo, t1 = hi, step = J.step;
    // scan points t_k = t0 + (k + 1/2) step with t_k < t1: k < (t1 - t0)/step - 1/2
    const double r = (t1 - t0) / step - 0.5;
    int kb = 0, ke = r > 0.0 ? (int)ceil(fmin(r, 2.0e9)) : 0;
    if (J.brick) {
        // a brick keeps the scan points inside its own box; neighbouring bricks
        // compute the shared crossing with the same expression, so every scan
        // point belongs to exactly one brick
        const double bl[3] = {(double)J.org[0], (double)J.org[1], (double)J.org[2]};
        const double bh[3] = {bl[0] + J.dims[0], bl[1] + J.dims[1], bl[2] + J.dims[2]};
        double blo, bhi;
        if (!slab(bl, bh, blo, bhi) || !(bhi > blo)) return false;
        kb = max(kb, (int)ceil(fmin(fmax((blo - t0) / step - 0.5, -1.0), 2.0e9)));
        ke = min(ke, (int)ceil(fmin(fmax((bhi - t0) / step - 0.5, -1.0), 2.0e9)));
    }
    // each plane keeps one interval of k: n.(o + t d) + d >= 0 is affine in t.
    // Bounds in closed form; a point this can misplace lies within FP64
    // rounding of the plane, far inside the decision margin
    for (int c = 0; c < J.n_clip; ++c) {
        const double* pl = J.clip[c];
        const double nd = pl[0] * d[0] + pl[1] * d[1] + pl[2] * d[2];
        const double no = pl[0] * o[0] + pl[1] * o[1] + pl[2] * o[2] + pl[3];
        if (nd == 0.0) {
            if (no < 0.0) ke = kb;
            continue;
        }
        const double kc = fmin(fmax((-no / nd - t0) / step - 0.5, -1.0), 2.0e9);
        if (nd > 0.0) kb = max(kb, (int)ceil(kc));          // kept for k >= kc
        else ke = min(ke, (int)floor(kc) + 1);              // kept for k <= kc
    }
    if (kb >= ke) return false;
    for (int a = 0; a < 3; ++a) {
        R.pb[a] = (float)(o[a] + t0 * d[a]);
        R.d[a] = (float)d[a];
    }
    R.kb = kb;
    R.ke = ke;
    R.t_first = (float)(t0 + ((double)kb + 0.5) * step);
    return true;
}

// One source at position p: nearest cell, or trilinear over the chain
// outputs of the 8 surrounding voxels (chain per fetched voxel, then blend).
template <int INTERP>
__device__ __forceinline__ float sample_source(const DevSource& S, const int dims[3], const float p[3]) {
    if (INTERP == 0) {
        const int qx = clampi((int)floorf(p[0]), 0, dims[0] - 1);
        const int qy = clampi((int)floorf(p[1]), 0, dims[1] - 1);
        const int qz = clampi((int)floorf(p[2]), 0, dims[2] - 1);
        const int off[1] = {qx * S.stride[0] + qy * S.stride[1] + qz * S.stride[2]};
        float v[1][4], r[1];
        fetch<1>(S, off, v);
        run_chain<1>(S, v, r);
        return r[0];
    }
    int i0[3], i1[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = p[a] - 0.5f;
        const float fl = floorf(u);
        w[a] = u - fl;
        i0[a] = (int)fl;
        i1[a] = i0[a] + 1;
        if (S.guard < 1) {
            i0[a] = clampi(i0[a], 0, dims[a] - 1);
            i1[a] = clampi(i1[a], 0, dims[a] - 1);
        }
    }
    const int x0 = i0[0] * S.stride[0], x1 = i1[0] * S.stride[0];
    const int y0 = i0[1] * S.stride[1], y1 = i1[1] * S.stride[1];
    const int z0 = i0[2] * S.stride[2], z1 = i1[2] * S.stride[2];
    const int off[8] = {x0 + y0 + z0, x1 + y0 + z0, x0 + y1 + z0, x1 + y1 + z0,
                        x0 + y0 + z1, x1 + y0 + z1, x0 + y1 + z1, x1 + y1 + z1};
    float v[8][4], c[8];
    fetch<8>(S, off, v);
    run_chain<8>(S, v, c);
    const float c00 = fmaf(w[0], c[1] - c[0], c[0]);
    const float c10 = fmaf(w[0], c[3] - c[2], c[2]);
    const float c01 = fmaf(w[0], c[5] - c[4], c[4]);
    const float c11 = fmaf(w[0], c[7] - c[6], c[6]);
    const float c0 = fmaf(w[1], c10 - c00, c00);
    const float c1 = fmaf(w[1], c11 - c01, c01);
    return fmaf(w[2], c1 - c0, c0);
}

// A plain source (packed FP32 scalar, no functor, guard layers: a derived
// component, or such a source itself) at position p: sample_source's loads
// and arithmetic, without its run-time storage and chain handling (and so
// without the registers they hold).
template <int INTERP>
__device__ __forceinline__ float sample_plain(const DevSource& S, const int dims[3], const float p[3]) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(S.base[0], S.num_records[0]);
    const int o = S.comp_off[0];
    if (INTERP == 0) {
        const int qx = clampi((int)floorf(p[0]), 0, dims[0] - 1);
        const int qy = clampi((int)floorf(p[1]), 0, dims[1] - 1);
        const int qz = clampi((int)floorf(p[2]), 0, dims[2] - 1);
        return ld_f32(r, qx * S.stride[0] + qy * S.stride[1] + qz * S.stride[2] + o);
    }
    int i0[3], i1[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = p[a] - 0.5f;
        const float fl = floorf(u);
        w[a] = u - fl;
        i0[a] = (int)fl;
        i1[a] = i0[a] + 1;
    }
    const int x0 = i0[0] * S.stride[0], x1 = i1[0] * S.stride[0];
    const int y0 = i0[1] * S.stride[1], y1 = i1[1] * S.stride[1];
    const int z0 = i0[2] * S.stride[2], z1 = i1[2] * S.stride[2];
    const int off[8] = {x0 + y0 + z0, x1 + y0 + z0, x0 + y1 + z0, x1 + y1 + z0,
                        x0 + y0 + z1, x1 + y0 + z1, x0 + y1 + z1, x1 + y1 + z1};
    float c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = ld_f32(r, off[i] + o);
    const float c00 = fmaf(w[0], c[1] - c[0], c[0]);
    const float c10 = fmaf(w[0], c[3] - c[2], c[2]);
    const float c01 = fmaf(w[0], c[5] - c[4], c[4]);
    const float c11 = fmaf(w[0], c[7] - c[6], c[6]);
    const float c0 = fmaf(w[1], c10 - c00, c00);
    const float c1 = fmaf(w[1], c11 - c01, c01);
    return fmaf(w[2], c1 - c0, c0);
}

template <int INTERP, bool PLAIN>
__device__ __forceinline__ float sample_any(const DevSource& S, const int dims[3], const float p[3]) {
    if constexpr (PLAIN) return sample_plain<INTERP>(S, dims, p);
    else return sample_source<INTERP>(S, dims, p);
}

// Compile-time source kinds of the specialized scan-point loop.
enum Kind : int { K_NONE = 0, K_F32x1 = 1, K_F32x3 = 2, K_F16x1 = 3, K_F16x3 = 4, K_BF16x1 = 5, K_BF16x3 = 6 };

template <int K> struct KindOf { static constexpr int dim = 1, dtype = DT_F32; };
template <> struct KindOf<K_F32x3> { static constexpr int dim = 3, dtype = DT_F32; };
template <> struct KindOf<K_F16x1> { static constexpr int dim = 1, dtype = DT_F16; };
template <> struct KindOf<K_F16x3> { static constexpr int dim = 3, dtype = DT_F16; };
template <> struct KindOf<K_BF16x1> { static constexpr int dim = 1, dtype = DT_BF16; };
template <> struct KindOf<K_BF16x3> { static constexpr int dim = 3, dtype = DT_BF16; };

// Voxel offsets of one source: nearest cell, or the 8 trilinear corners with
// the border clamp of guard-less sources.  24-bit multiplies (the host admits
// a signature only when every stride is below 2^23 bytes).
template <int INTERP, bool CLAMP = true>
__device__ __forceinline__ void corner_offsets(const DevSource& S, const int dims[3], const int (&i0)[3],
                                               int (&off)[INTERP ? 8 : 1]) {
    if (INTERP == 0) {
        off[0] = __mul24(i0[0], S.stride[0]) + __mul24(i0[1], S.stride[1]) + __mul24(i0[2], S.stride[2]);
        return;
    }
    int a0[3], a1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        a0[a] = i0[a];
        a1[a] = i0[a] + 1;
        if (CLAMP && S.guard < 1) {
            a0[a] = clampi(a0[a], 0, dims[a] - 1);
            a1[a] = clampi(a1[a], 0, dims[a] - 1);
        }
    }
    const int x0 = __mul24(a0[0], S.stride[0]), x1 = __mul24(a1[0], S.stride[0]);
    const int y0 = __mul24(a0[1], S.stride[1]), y1 = __mul24(a1[1], S.stride[1]);
    const int z0 = __mul24(a0[2], S.stride[2]), z1 = __mul24(a1[2], S.stride[2]);
    off[0] = x0 + y0 + z0;
    off[1] = x1 + y0 + z0;
    off[2] = x0 + y1 + z0;
    off[3] = x1 + y1 + z0;
    off[4] = x0 + y0 + z1;
    off[5] = x1 + y0 + z1;
    off[6] = x0 + y1 + z1;
    off[7] = x1 + y1 + z1;
}

template <int K, int N>
__device__ __forceinline__ void fetch_kind(const DevSource& S, const int (&off)[N], float (&v)[N][4]) {
    constexpr int D = KindOf<K>::dim, T = KindOf<K>::dtype;
    const __amdgpu_buffer_rsrc_t r = make_rsrc(S.base[0], S.num_records[0]);
    const int o = S.comp_off[0];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[i][c] = 0.f;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            if (T == DT_F32) v[i][c] = ld_f32(r, off[i] + o + 4 * c);
            else v[i][c] = ld_scalar(r, off[i] + o + 2 * c, T);
        }
    }
}

// The 8 trilinear corners (or the nearest cell) of a three-source derived
// volume, 12-byte records, same corner order as corner_offsets.
// PAIRED (layout 1, (y, z) pairs): the x + 1 corners are 48 bytes on (the
// loads' scalar offset); the y + 1 and z + 1 corners lie in the same pair or
// the next one depending on the parity of the index.  A wave's gathers of one
// corner touch fewer cache lines on oblique rays than in the x-fastest layout.
// Layout 0 (x fastest): two per-lane base offsets (z0 and z1 planes) and the
// wave-uniform x/y corner steps in the scalar offset.
template <int INTERP, bool PAIRED>
__device__ __forceinline__ void fetch_il3(const DevSource& S, const int (&i0)[3], float (&v)[INTERP ? 8 : 1][4]) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(S.base[0], S.num_records[0]);
    const int sx = __builtin_amdgcn_readfirstlane(S.stride[0]);
    const int sy = __builtin_amdgcn_readfirstlane(S.stride[1]);
    const int sz = __builtin_amdgcn_readfirstlane(S.stride[2]);
    auto ld3 = [&](int vo, int so, float (&d)[4]) {
        d[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
        d[1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo + 4, so, 0));
        d[2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo + 8, so, 0));
        d[3] = 0.f;
    };
    if constexpr (PAIRED) {
        const int yl = i0[1] & 1, zl = i0[2] & 1;
        const int b0 = __mul24(i0[2] >> 1, sz) + __mul24(i0[1] >> 1, sy) + __mul24(i0[0], sx) + __mul24(zl, 24) +
                       __mul24(yl, 12) + S.comp_off[0];
        if constexpr (INTERP == 0) {
            ld3(b0, 0, v[0]);
        } else {
            const int oy = __mul24(yl, sy - 24) + 12;   // y + 1: same pair (+12) or the next one
            const int oz = __mul24(zl, sz - 48) + 24;   // z + 1: same pair (+24) or the next one
            const int b2 = b0 + oy, b4 = b0 + oz, b6 = b4 + oy;
            ld3(b0, 0, v[0]);
            ld3(b0, sx, v[1]);
            ld3(b2, 0, v[2]);
            ld3(b2, sx, v[3]);
            ld3(b4, 0, v[4]);
            ld3(b4, sx, v[5]);
            ld3(b6, 0, v[6]);
            ld3(b6, sx, v[7]);
        }
    } else {
        const int b0 = __mul24(i0[0], sx) + __mul24(i0[1], sy) + __mul24(i0[2], sz) + S.comp_off[0];
        if constexpr (INTERP == 0) {
            ld3(b0, 0, v[0]);
        } else {
            const int b1 = b0 + sz;
            ld3(b0, 0, v[0]);
            ld3(b0, sx, v[1]);
            ld3(b0, sy, v[2]);
            ld3(b0, sx + sy, v[3]);
            ld3(b1, 0, v[4]);
            ld3(b1, sx, v[5]);
            ld3(b1, sy, v[6]);
            ld3(b1, sx + sy, v[7]);
        }
    }
}

template <int N>
__device__ __forceinline__ float blend(const float (&c)[N], const float (&w)[3]) {
    if (N == 1) return c[0];
    const float c00 = fmaf(w[0], c[1] - c[0], c[0]);
    const float c10 = fmaf(w[0], c[3] - c[2], c[2]);
    const float c01 = fmaf(w[0], c[5] - c[4], c[4]);
    const float c11 = fmaf(w[0], c[7] - c[6], c[6]);
    const float c0 = fmaf(w[1], c10 - c00, c00);
    const float c1 = fmaf(w[1], c11 - c01, c01);
    return fmaf(w[2], c1 - c0, c0);
}

// ---------------------------------------------------------------------------
// Scan points.  point_generic evaluates one scan point with the runtime
// source loop (any sources); points<...> evaluates U consecutive scan points
// for a compile-time source signature, issuing every load before any is
// consumed (the source loop unrolled at compile time, as the paper does with
// template metaprogramming, Sec. 3.2).  Both return the mixed premultiplied
// colour E and opacity S of each point and round alike at every step (the
// trilinear cell coordinates come from point_at and a subtraction of 1/2 in
// one, from cell_at in the other, which give the same numbers), so they give
// the same image bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mix_finish(float& S, float (&E)[3]) {
    if (S > 1.f) {
        const float inv = 1.f / S;
        E[0] *= inv;
        E[1] *= inv;
        E[2] *= inv;
        S = 1.f;
    }
}

template <int INTERP>
__device__ __forceinline__ void point_generic(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                              int k, float (&E)[3], float& S) {
    const float tk = ((float)k + 0.5f) * (float)J.step;
    float p[3];
    point_at(J, R, tk, p);
    const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
    S = 0.f;
    E[0] = E[1] = E[2] = 0.f;
    for (int s = 0; s < J.n_src; ++s) {
        const DevSource& src = J.src[s];
        const float x = sample_source<INTERP>(src, dims, p);
        const float4 c = classify(s_tf + s * kTfLds, x);
        const float wa = src.weight * c.w;
        S = fmaf(src.weight, c.w, S);
        E[0] = fmaf(wa, c.x, E[0]);
        E[1] = fmaf(wa, c.y, E[1]);
        E[2] = fmaf(wa, c.z, E[2]);
    }
    mix_finish(S, E);
}

template <int SIG> struct SigKinds { static constexpr int k0 = K_NONE, k1 = K_NONE, k2 = K_NONE; };
template <> struct SigKinds<SIG_F32x1> { static constexpr int k0 = K_F32x1, k1 = K_NONE, k2 = K_NONE; };
template <> struct SigKinds<SIG_PIC3_F32> { static constexpr int k0 = K_F32x1, k1 = K_F32x3, k2 = K_F32x3; };
template <> struct SigKinds<SIG_PIC3_F16> { static constexpr int k0 = K_F16x1, k1 = K_F16x3, k2 = K_F16x3; };
template <> struct SigKinds<SIG_PIC3_BF16> { static constexpr int k0 = K_BF16x1, k1 = K_BF16x3, k2 = K_BF16x3; };
template <> struct SigKinds<SIG_IL3> { static constexpr int k0 = K_F32x1, k1 = K_F32x1, k2 = K_F32x1; };
template <> struct SigKinds<SIG_IL3P> { static constexpr int k0 = K_F32x1, k1 = K_F32x1, k2 = K_F32x1; };

// PS (per source): load, chain, blend and classify one source before the
// next one's loads; fewer live registers (more resident waves) at the cost of
// one memory round trip per source.  Same arithmetic either way.
template <int INTERP, int U, int SIG, bool PS>
__device__ __forceinline__ void points(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R, int k,
                                       float (&E)[U][3], float (&S)[U]) {
    if constexpr (SIG == SIG_GENERIC) {
        static_assert(U == 1, "the generic loop evaluates one scan point at a time");
        point_generic<INTERP>(J, s_tf, R, k, E[0], S[0]);
    } else {
        constexpr int K0 = SigKinds<SIG>::k0, K1 = SigKinds<SIG>::k1, K2 = SigKinds<SIG>::k2;
        constexpr int KS[3] = {K0, K1, K2};
        constexpr int NV = INTERP ? 8 : 1;
        constexpr int NS = (K0 != K_NONE) + (K1 != K_NONE) + (K2 != K_NONE);
        // the host admits the three-source signatures only with guard layers: no border clamp
        constexpr bool CL = SIG == SIG_F32x1;
        const float step = (float)J.step;
        const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
        int i0[U][3];
        float wts[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = min(k + u, R.ke - 1);
            float p[3];
            if (INTERP == 0) point_at(J, R, ((float)kk + 0.5f) * step, p);
            else cell_at(J, R, kk, p);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (INTERP == 0) {
                    i0[u][a] = clampi((int)floorf(p[a]), 0, dims[a] - 1);
                    wts[u][a] = 0.f;
                } else {
                    const float fl = floorf(p[a]);
                    wts[u][a] = p[a] - fl;
                    i0[u][a] = (int)fl;
                }
            }
            S[u] = 0.f;
            E[u][0] = E[u][1] = E[u][2] = 0.f;
        }
        auto accumulate = [&](int u, int s, float x) {
            const float4 cl = classify(s_tf + s * kTfLds, x);
            const float wa = J.src[s].weight * cl.w;
            S[u] = fmaf(J.src[s].weight, cl.w, S[u]);
            E[u][0] = fmaf(wa, cl.x, E[u][0]);
            E[u][1] = fmaf(wa, cl.y, E[u][1]);
            E[u][2] = fmaf(wa, cl.z, E[u][2]);
        };
        if constexpr (SIG == SIG_IL3 || SIG == SIG_IL3P) {
            // the three chain outputs of a voxel are adjacent: one 12-byte load per corner
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float v[NV][4];
                fetch_il3<INTERP, SIG == SIG_IL3P>(J.src[0], i0[u], v);
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    float c[NV];
#pragma unroll
                    for (int i = 0; i < NV; ++i) c[i] = v[i][s];
                    accumulate(u, s, blend<NV>(c, wts[u]));
                }
            }
        } else if constexpr (PS) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int off[NV];
                    float v[NV][4], c[NV];
                    corner_offsets<INTERP, CL>(J.src[s], dims, i0[u], off);
                    if (s == 0) fetch_kind<KS[0], NV>(J.src[0], off, v);
                    else if (s == 1) fetch_kind<KS[1], NV>(J.src[1], off, v);
                    else fetch_kind<KS[2], NV>(J.src[2], off, v);
                    if (s == 0) run_chain<NV, KindOf<KS[0]>::dim>(J.src[0], v, c);
                    else if (s == 1) run_chain<NV, KindOf<KS[1]>::dim>(J.src[1], v, c);
                    else run_chain<NV, KindOf<KS[2]>::dim>(J.src[2], v, c);
                    accumulate(u, s, blend<NV>(c, wts[u]));
                }
            }
        } else {
            // every load of U scan points first, then chains, interpolation, classification
            float vals[U][3][NV][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int off[NV];
                if (NS > 0) {
                    corner_offsets<INTERP, CL>(J.src[0], dims, i0[u], off);
                    fetch_kind<K0, NV>(J.src[0], off, vals[u][0]);
                }
                if (NS > 1) {
                    corner_offsets<INTERP, CL>(J.src[1], dims, i0[u], off);
                    fetch_kind<K1, NV>(J.src[1], off, vals[u][1]);
                }
                if (NS > 2) {
                    corner_offsets<INTERP, CL>(J.src[2], dims, i0[u], off);
                    fetch_kind<K2, NV>(J.src[2], off, vals[u][2]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    float c[NV];
                    if (s == 0) run_chain<NV, KindOf<KS[0]>::dim>(J.src[0], vals[u][0], c);
                    else if (s == 1) run_chain<NV, KindOf<KS[1]>::dim>(J.src[1], vals[u][1], c);
                    else run_chain<NV, KindOf<KS[2]>::dim>(J.src[2], vals[u][2], c);
                    accumulate(u, s, blend<NV>(c, wts[u]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) mix_finish(S[u], E[u]);
    }
}

// One lane per ray: classical front-to-back compositing, U scan points per
// step, early termination at the first point whose opacity reaches ert.
template <int INTERP, int U, int SIG, bool PS>
__device__ __forceinline__ void march_seq(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                          float4& out, int& count) {
    const float ert = J.ert;
    float Cr = 0.f, Cg = 0.f, Cb = 0.f, A = 0.f;
    int n = 0;
    bool done = false;
    for (int k = R.kb; k < R.ke && !done; k += U) {
        float E[U][3], S[U];
        points<INTERP, U, SIG, PS>(J, s_tf, R, k, E, S);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k + u < R.ke && !done) {
                const float T = 1.f - A;
                Cr = fmaf(T, E[u][0], Cr);
                Cg = fmaf(T, E[u][1], Cg);
                Cb = fmaf(T, E[u][2], Cb);
                A = fmaf(T, S[u], A);
                ++n;
                if (A >= ert) done = true;
            }
        }
    }
    out = make_float4(Cr, Cg, Cb, A);
    count = n;
}

// Value of the lane D below inside a row of 16 lanes (DPP row_shr:D); a lane
// whose source would lie in another row reads 0.
template <int D>
__device__ __forceinline__ float lane_up(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x110 + D, 0xF, 0xF,
                                                                 true));
}

// Running front-to-back state of one ray composited by a group of G lanes.
struct RayAccum {
    float C0, C1, C2, A;
    int n;
};

// Composite one row of G scan points (k0 .. k0+G-1; lane g holds point
// k0 + g, `valid` when below R.ke) into acc: an inclusive scan of the
// front-to-back operator across the group, then termination at the first
// point whose cumulative opacity reaches ert.  Returns true when the ray is
// finished (termination, or no scan point left).
// Inclusive scan of the front-to-back operator over the G lanes of a group
// (lane g ends with the composite of lanes 0..g, lane 0 frontmost).
template <int G>
__device__ __forceinline__ void group_scan(int lane, float& c0, float& c1, float& c2, float& a) {
    const int g = lane & (G - 1);
    // inclusive scan inside each row of 16 lanes ...
#pragma unroll
    for (int d = 1; d < (G < 16 ? G : 16); d <<= 1) {
        float o0, o1, o2, oa;
        if (d == 1) {
            o0 = lane_up<1>(c0); o1 = lane_up<1>(c1); o2 = lane_up<1>(c2); oa = lane_up<1>(a);
        } else if (d == 2) {
            o0 = lane_up<2>(c0); o1 = lane_up<2>(c1); o2 = lane_up<2>(c2); oa = lane_up<2>(a);
        } else if (d == 4) {
            o0 = lane_up<4>(c0); o1 = lane_up<4>(c1); o2 = lane_up<4>(c2); oa = lane_up<4>(a);
        } else {
            o0 = lane_up<8>(c0); o1 = lane_up<8>(c1); o2 = lane_up<8>(c2); oa = lane_up<8>(a);
        }
        // with whole rows per group the shifted-in value of a row's first lanes
        // is 0 (bound_ctrl), the identity of the operator: no mask needed
        if (G >= 16 || (g & 15) >= d) {
            const float t = 1.f - oa;
            c0 = fmaf(t, c0, o0);
            c1 = fmaf(t, c1, o1);
            c2 = fmaf(t, c2, o2);
            a = fmaf(t, a, oa);
        }
    }
    // ... then each row appends the total of the rows before it in its group
    // (the last lane of the row below, after that row's own update)
#pragma unroll
    for (int r = 16; r < G; r <<= 1) {
        const int src = (lane & ~(2 * r - 1)) + r - 1;
        const float o0 = __shfl(c0, src, 64), o1 = __shfl(c1, src, 64), o2 = __shfl(c2, src, 64);
        const float oa = __shfl(a, src, 64);
        if (g & r) {
            const float t = 1.f - oa;
            c0 = fmaf(t, c0, o0);
            c1 = fmaf(t, c1, o1);
            c2 = fmaf(t, c2, o2);
            a = fmaf(t, a, oa);
        }
    }
}

// One row of G scan points of a ray composited into acc.  A lane past the ray's
// last scan point (valid false) may carry any finite values (the callers give it
// the last point's sample): the scan is inclusive, so no kept lane's prefix
// depends on it, the termination ballot masks it, and the lane taken is never
// past the row's last kept point.
template <int G>
__device__ __forceinline__ bool row_composite(const DevJob& J, const RaySetup& R, int lane, int k0, bool valid,
                                              float c0, float c1, float c2, float a, RayAccum& acc) {
    group_scan<G>(lane, c0, c1, c2, a);
    const float T = 1.f - acc.A;
    const float n0 = fmaf(T, c0, acc.C0), n1 = fmaf(T, c1, acc.C1), n2 = fmaf(T, c2, acc.C2), na = fmaf(T, a, acc.A);
    const unsigned long long m = __builtin_amdgcn_ballot_w64(na >= J.ert) & __builtin_amdgcn_ballot_w64(valid);
    constexpr unsigned long long kGroupMask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull);
    const unsigned long long bits = (m >> (lane & ~(G - 1))) & kGroupMask;
    const bool stop = bits != 0;
    // the first terminating point, else the row's last kept one (k0 < R.ke, so
    // last >= 0; every set bit belongs to a kept point, i.e. lies at or below last)
    const int last = min(G, R.ke - k0) - 1;
    int sel;
    if constexpr (G <= 32) sel = __builtin_ctz((unsigned)bits | (1u << last));
    else sel = __builtin_ctzll(bits | (1ull << last));
    acc.n += sel + 1;
    acc.C0 = __shfl(n0, sel, G);
    acc.C1 = __shfl(n1, sel, G);
    acc.C2 = __shfl(n2, sel, G);
    acc.A = __shfl(na, sel, G);
    return stop || k0 + G >= R.ke;
}

// One row of the lanes-per-ray schedule: scan points k0 .. k0+G-1 (those
// below R.ke), composited into acc.  Returns true when the ray is finished.
template <int INTERP, int G, int SIG, bool PS>
__device__ __forceinline__ bool lanes_row(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                          int lane, int k0, RayAccum& acc) {
    const int g = lane & (G - 1);
    const int k = k0 + g;
    const bool valid = k < R.ke;
    float E[1][3], S[1];
    points<INTERP, 1, SIG, PS>(J, s_tf, R, valid ? k : R.ke - 1, E, S);
    return row_composite<G>(J, R, lane, k0, valid, E[0][0], E[0][1], E[0][2], S[0], acc);
}

// Interleaved derived volume (SIG_IL3), G lanes per ray, software-pipelined:
// the corner loads of a lane's next scan point are issued before the current
// one is blended, classified and composited, so a row's memory latency
// overlaps the previous row's arithmetic.  The arithmetic is that of
// lanes_row, operation for operation.
template <int INTERP>
__device__ __forceinline__ void il3_locate(const DevJob& J, const RaySetup& R, int k, int (&i0)[3], float (&w)[3]) {
    const int kk = min(k, R.ke - 1);
    float p[3];
    if (INTERP == 0) point_at(J, R, ((float)kk + 0.5f) * (float)J.step, p);
    else cell_at(J, R, kk, p);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (INTERP == 0) {
            i0[a] = clampi((int)floorf(p[a]), 0, J.dims[a] - 1);
            w[a] = 0.f;
        } else {
            const float fl = floorf(p[a]);
            w[a] = p[a] - fl;
            i0[a] = (int)fl;
        }
    }
}

template <int NV>
__device__ __forceinline__ void il3_mix(const DevJob& J, const float4* __restrict__ s_tf, const float (&v)[NV][4],
                                        const float (&w)[3], float (&E)[3], float& S) {
    S = 0.f;
    E[0] = E[1] = E[2] = 0.f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        float c[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) c[i] = v[i][s];
        const float4 cl = classify(s_tf + s * kTfLds, blend<NV>(c, w));
        const float wa = J.src[s].weight * cl.w;
        S = fmaf(J.src[s].weight, cl.w, S);
        E[0] = fmaf(wa, cl.x, E[0]);
        E[1] = fmaf(wa, cl.y, E[1]);
        E[2] = fmaf(wa, cl.z, E[2]);
    }
    mix_finish(S, E);
}

template <int INTERP, int G, bool PAIRED>
__device__ __forceinline__ void march_lanes_il3(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                                int lane, float4& out, int& count) {
    constexpr int NV = INTERP ? 8 : 1;
    const int g = lane & (G - 1);
    int i0[3];
    float w[3], v[NV][4];
    il3_locate<INTERP>(J, R, R.kb + g, i0, w);
    fetch_il3<INTERP, PAIRED>(J.src[0], i0, v);
    RayAccum acc = {0.f, 0.f, 0.f, 0.f, 0};
    for (int k0 = R.kb;; k0 += G) {
        // the next row's loads (clamped to the last scan point: always in bounds)
        int i0n[3];
        float wn[3], vn[NV][4];
        il3_locate<INTERP>(J, R, k0 + G + g, i0n, wn);
        fetch_il3<INTERP, PAIRED>(J.src[0], i0n, vn);
        const bool valid = k0 + g < R.ke;
        float E[3], S;
        il3_mix<NV>(J, s_tf, v, w, E, S);
        if (row_composite<G>(J, R, lane, k0, valid, E[0], E[1], E[2], S, acc))
            break;
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[i][c] = vn[i][c];
        w[0] = wn[0];
        w[1] = wn[1];
        w[2] = wn[2];
    }
    out = make_float4(acc.C0, acc.C1, acc.C2, acc.A);
    count = acc.n;
}

// G lanes per ray: lane g evaluates scan points kb + g, kb + g + G, ...; each
// row of G points is composited in order with an inclusive scan of the
// associative front-to-back operator (C, A) o (C', A') = (C + (1-A) C',
// A + (1-A) A') across the group, then appended to the ray's running state.
// The first point whose cumulative opacity reaches ert ends the ray, exactly
// where the one-lane loop would stop.
template <int INTERP, int G, int SIG, bool PS>
__device__ __forceinline__ void march_lanes(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                            int lane, float4& out, int& count) {
    RayAccum acc = {0.f, 0.f, 0.f, 0.f, 0};
    for (int k0 = R.kb;; k0 += G)
        if (lanes_row<INTERP, G, SIG, PS>(J, s_tf, R, lane, k0, acc)) break;
    out = make_float4(acc.C0, acc.C1, acc.C2, acc.A);
    count = acc.n;
}

template <int INTERP, int U, int G, int SIG, bool PS>
__device__ __forceinline__ void march_sig(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                          int lane, float4& out, int& count) {
    if constexpr (G == 1) march_seq<INTERP, (SIG == SIG_GENERIC ? 1 : U), SIG, PS>(J, s_tf, R, out, count);
    else if constexpr ((SIG == SIG_IL3 || SIG == SIG_IL3P) && !PS)
        march_lanes_il3<INTERP, G, SIG == SIG_IL3P>(J, s_tf, R, lane, out, count);
    else march_lanes<INTERP, G, SIG, PS>(J, s_tf, R, lane, out, count);
}

template <int INTERP, int U, int G, bool PS>
__device__ __forceinline__ void march_dispatch(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                               int lane, float4& out, int& count) {
    switch (J.sig) {
    case SIG_F32x1: march_sig<INTERP, U, G, SIG_F32x1, PS>(J, s_tf, R, lane, out, count); break;
    case SIG_PIC3_F32: march_sig<INTERP, U, G, SIG_PIC3_F32, PS>(J, s_tf, R, lane, out, count); break;
    case SIG_PIC3_F16: march_sig<INTERP, U, G, SIG_PIC3_F16, PS>(J, s_tf, R, lane, out, count); break;
    case SIG_PIC3_BF16: march_sig<INTERP, U, G, SIG_PIC3_BF16, PS>(J, s_tf, R, lane, out, count); break;
    case SIG_IL3: march_sig<INTERP, U, G, SIG_IL3, PS>(J, s_tf, R, lane, out, count); break;
    case SIG_IL3P: march_sig<INTERP, U, G, SIG_IL3P, PS>(J, s_tf, R, lane, out, count); break;
    default: march_sig<INTERP, U, G, SIG_GENERIC, PS>(J, s_tf, R, lane, out, count); break;
    }
}

// Iso-surface mode (a listed feature, Sec. 3; the paper gives no algorithm):
// the first place where a source's interpolated chain output crosses its iso
// value between two consecutive scan points, placed by linear interpolation
// between them; opaque, coloured by the source's table at the iso value and
// lit by a headlight, 0.3 + 0.7 |cos| of the angle between the ray and the
// central-difference gradient (half a voxel each side).  One lane per ray;
// the source loop is uniform, so every source's buffer resource stays scalar.
// The crossing of source s between scan points k - 1 and k, at fraction f of
// the step: opaque, the source's table colour at its iso value lit by a
// headlight from the central-difference gradient (half a voxel each side).
// s must be wave-uniform (the source's buffer resource is scalar).
template <int INTERP, bool PLAIN>
__device__ __forceinline__ float4 iso_shade(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                            int s, int k, float f) {
    // no contraction: (k + 1/2) step - tp is rounded as written wherever this is inlined
#pragma clang fp contract(off)
    const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
    const float step = (float)J.step;
    const DevSource& S = J.src[s];
    const float tp = ((float)(k - 1) + 0.5f) * step;
    const float ts = fmaf(f, ((float)k + 0.5f) * step - tp, tp);
    float q[3];
    point_at(J, R, ts, q);
    float g[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {           // one axis at a time keeps register use low
        const float hx = a == 0 ? 0.5f : 0.f, hy = a == 1 ? 0.5f : 0.f, hz = a == 2 ? 0.5f : 0.f;
        const float qp[3] = {q[0] + hx, q[1] + hy, q[2] + hz}, qm[3] = {q[0] - hx, q[1] - hy, q[2] - hz};
        const float d = sample_any<INTERP, PLAIN>(S, dims, qp) - sample_any<INTERP, PLAIN>(S, dims, qm);
        g[0] = a == 0 ? d : g[0];
        g[1] = a == 1 ? d : g[1];
        g[2] = a == 2 ? d : g[2];
    }
    const float gl = sqrtf(fmaf(g[0], g[0], fmaf(g[1], g[1], g[2] * g[2])));
    const float cosine = gl > 0.f ? fabsf(fmaf(g[0], R.d[0], fmaf(g[1], R.d[1], g[2] * R.d[2]))) / gl : 1.f;
    const float light = fmaf(0.7f, fminf(cosine, 1.f), 0.3f);
    const float4 c = classify(s_tf + s * kTfLds, S.iso);
    return make_float4(c.x * light, c.y * light, c.z * light, 1.f);
}

// One lane per ray: scan points in order, every source at each, until the
// first crossing.
template <int INTERP, bool PLAIN>
__device__ __forceinline__ void march_iso(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R,
                                          float4& out, int& count) {
    const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
    const float step = (float)J.step;
    float prev[kMaxSources];
    int hit = -1, n = 0, k = R.kb;
    float f = 0.f;
    for (; k < R.ke; ++k) {
        float p[3];
        point_at(J, R, ((float)k + 0.5f) * step, p);
        ++n;
        for (int s = 0; s < J.n_src; ++s) {
            const DevSource& S = J.src[s];
            const float x = sample_any<INTERP, PLAIN>(S, dims, p);
            if (hit < 0 && k > R.kb && ((prev[s] >= S.iso) != (x >= S.iso))) {
                hit = s;
                f = (S.iso - prev[s]) / (x - prev[s]);
            }
            prev[s] = x;
        }
        if (hit >= 0) break;
    }
    out = make_float4(0.f, 0.f, 0.f, 0.f);
    count = n;
    // shade, one source at a time over the lanes whose surface it is
    for (int s = 0; s < J.n_src; ++s)
        if (hit == s) out = iso_shade<INTERP, PLAIN>(J, s_tf, R, s, k, f);
}

// G lanes per ray: lane g takes scan point k0 + g of each row of G points; its
// predecessor's values come from lane g - 1 (lane 0: the last point of the row
// before), so every lane tests its own pair of consecutive points at once and
// the ray's crossing is the first lane (then the first source in index order)
// that sees one: the point, source and fraction the one-lane loop finds, with
// the same arithmetic, in a fraction of its dependent steps.  The crossing's
// lane shades, and passes colour and count to the group's first lane.
template <int INTERP, int G, bool PLAIN>
__device__ __forceinline__ void march_iso_lanes(const DevJob& J, const float4* __restrict__ s_tf,
                                                const RaySetup& R, int lane, float4& out, int& count) {
    const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
    const float step = (float)J.step;
    const int g = lane & (G - 1), base = lane & ~(G - 1);
    constexpr unsigned long long kGroupMask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull);
    float carry[kMaxSources] = {};              // values at the last point of the previous row
    int sel = -1, my_s = -1, k = R.kb;
    float my_f = 0.f;
    for (int k0 = R.kb;; k0 += G) {
        k = k0 + g;
        const bool valid = k < R.ke;
        float p[3];
        point_at(J, R, ((float)(valid ? k : R.ke - 1) + 0.5f) * step, p);
        for (int s = 0; s < J.n_src; ++s) {
            const DevSource& S = J.src[s];
            const float x = sample_any<INTERP, PLAIN>(S, dims, p);
            float prev = __shfl(x, base + ((g + G - 1) & (G - 1)), 64);
            if (g == 0) prev = carry[s];
            if (my_s < 0 && valid && k > R.kb && ((prev >= S.iso) != (x >= S.iso))) {
                my_s = s;
                my_f = (S.iso - prev) / (x - prev);
            }
            carry[s] = __shfl(x, base + G - 1, 64);
        }
        const unsigned long long bits = (__builtin_amdgcn_ballot_w64(my_s >= 0) >> base) & kGroupMask;
        if (bits) {
            sel = (int)__builtin_ctzll(bits);
            count = k0 + sel - R.kb + 1;
            break;
        }
        if (k0 + G >= R.ke) {
            count = R.ke - R.kb;
            break;
        }
    }
    // shade one source at a time: the source must be the same on every active lane
    // (its buffer resource is read as wave-uniform), whatever surface each ray found
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int s = 0; s < J.n_src; ++s)
        if (g == sel && my_s == s) c = iso_shade<INTERP, PLAIN>(J, s_tf, R, s, k, my_f);
    const int src = base + (sel >= 0 ? sel : 0);
    out = make_float4(__shfl(c.x, src, 64), __shfl(c.y, src, 64), __shfl(c.z, src, 64), __shfl(c.w, src, 64));
}

__device__ __forceinline__ int find_job(const DevJob* __restrict__ jobs, int n_jobs, int tile) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Pixel of this lane in tile t of job J (G lanes share one ray); false
// outside the image.
template <int G>
__device__ __forceinline__ bool pixel_of(const DevJob& J, int t, int lane, int wave, int& px, int& py) {
    const int ray = lane / G;
    const int ww = J.wave_w, wh = (64 / G) / ww;
    const int gx = J.waves_x, gy = 4 / gx;
    const int tx = t % J.tiles_x, ty = t / J.tiles_x;
    px = J.cull[0] + tx * (ww * gx) + (wave % gx) * ww + ray % ww;
    py = J.cull[1] + ty * (wh * gy) + (wave / gx) * wh + ray / ww;
    return px <= J.cull[2] && py <= J.cull[3];
}

// Waves-per-SIMD hint: W = 0 leaves register allocation to the compiler and
// issues every load of a scan point at once; W > 0 asks for at least W
// resident waves per SIMD and evaluates the sources one after another.
// SIGK >= 0: the kernel runs only that source signature (every job of the
// launch has it); SIGK = -1: it dispatches on each job's signature; SIGK = -2:
// iso-surface jobs; SIGK = -3: iso-surface jobs whose sources are all plain
// (sample_plain).
template <int U, int G, int W, int SIGK>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1, 8)))
void raycast_kernel(const DevJob* __restrict__ jobs, const float4* __restrict__ tf_pool, int* __restrict__ cursor,
                    int n_jobs, int total_tiles, int persistent) {
    extern __shared__ float4 s_tf[];
    __shared__ int s_tile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int cur_job = -1;
    for (int iter = 0;; ++iter) {
        int tile;
        if (persistent) {
            if (threadIdx.x == 0) s_tile = atomicAdd(cursor, 1);
            __syncthreads();
            tile = s_tile;
            __syncthreads();
            if (tile >= total_tiles) break;
        } else {
            if (iter > 0) break;
            tile = (int)blockIdx.x;
        }
        tile = __builtin_amdgcn_readfirstlane(tile);
        const int job = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, tile));
        const DevJob& J = jobs[job];
        // tiles cover the box's screen rectangle only (the fill kernel clears the rest)
        int px = 0, py = 0;
        const bool in_image = pixel_of<G>(J, tile - J.tile_begin, lane, wave, px, py);
        RaySetup R;
        bool hit;
        if (J.rays) {
            // set up by the prepass, one lane per ray
            hit = false;
            if (in_image) {
                const int rw = J.cull[2] - J.cull[0] + 1;
                const RayRec& rr = static_cast<const RayRec*>(J.rays)[(py - J.cull[1]) * rw + (px - J.cull[0])];
                R.kb = rr.kb;
                R.ke = rr.ke;
                hit = R.kb < R.ke;
                if (hit) {
                    for (int a = 0; a < 3; ++a) {
                        R.pb[a] = rr.pb[a];
                        R.d[a] = rr.d[a];
                    }
                    R.t_first = rr.t_first;
                }
            }
        } else {
            hit = in_image && setup_ray(J, px, py, R);
        }
        // tiles no ray of which meets the box skip the transfer tables; the
        // barrier also ends every read of the previous tile's tables
        if (__syncthreads_or(hit) && job != cur_job) {
            const int n = J.n_src * kTfLds;
            for (int i = threadIdx.x; i < n; i += kBlockThreads) {
                const int s = i / kTfLds, e = min(i % kTfLds, kTfEntries - 1);
                s_tf[i] = tf_pool[(size_t)J.src[s].tf_slot * kTfRows + 2 * e];
            }
            __syncthreads();
            cur_job = job;
        }
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        int count = 0;
        if (hit) {
            if constexpr ((SIGK == -2 || SIGK == -3) && G == 1) {
                constexpr bool PL = SIGK == -3;
                if (J.interp) march_iso<1, PL>(J, s_tf, R, c, count);
                else march_iso<0, PL>(J, s_tf, R, c, count);
            } else if constexpr (SIGK == -2 || SIGK == -3) {
                constexpr bool PL = SIGK == -3;
                if (J.interp) march_iso_lanes<1, G, PL>(J, s_tf, R, lane, c, count);
                else march_iso_lanes<0, G, PL>(J, s_tf, R, lane, c, count);
            } else if constexpr (SIGK < 0) {
                if (J.interp) march_dispatch<1, U, G, (W > 0)>(J, s_tf, R, lane, c, count);
                else march_dispatch<0, U, G, (W > 0)>(J, s_tf, R, lane, c, count);
            } else {
                if (J.interp) march_sig<1, U, G, SIGK, (W > 0)>(J, s_tf, R, lane, c, count);
                else march_sig<0, U, G, SIGK, (W > 0)>(J, s_tf, R, lane, c, count);
            }
        }
        if (in_image && (lane & (G - 1)) == 0) {
            const size_t pix = (size_t)py * J.width + px;
            reinterpret_cast<float4*>(J.out)[pix] = c;
            if (J.out_samples) J.out_samples[pix] = count;
            if (J.out_depth) J.out_depth[pix] = hit ? R.t_first : __builtin_inff();
        }
    }
}

// ---------------------------------------------------------------------------
// Pooled schedule (one job).  ray_setup_kernel sets up every pixel's ray and
// appends the rays that keep scan points to a compact list (the others get
// their empty output at once); raycast_pool_kernel keeps its waves resident
// and hands the listed rays to groups of G lanes as groups free up, so a
// wave's lanes stay busy whatever the lengths of its rays.  Each ray is
// composited row by row exactly as in the tiled schedule with G lanes per ray.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ray_setup_kernel(const DevJob* __restrict__ jobs, RayRec* __restrict__ rays,
                                                        int* __restrict__ counters) {
    const DevJob& J = jobs[0];
    const int px = (int)(blockIdx.x * 16 + (threadIdx.x & 15));
    const int py = (int)(blockIdx.y * 16 + (threadIdx.x >> 4));
    const bool in_image = px < J.width && py < J.height;
    const bool in_rect = px >= J.cull[0] && px <= J.cull[2] && py >= J.cull[1] && py <= J.cull[3];
    RaySetup R;
    const bool hit = in_image && in_rect && setup_ray(J, px, py, R);
    // one append per wave
    const unsigned long long m = __ballot(hit);
    const int lane = (int)(threadIdx.x & 63);
    int base = 0;
    if (m) {
        const int first = __builtin_ctzll(m);
        if (lane == first) base = atomicAdd(&counters[0], __popcll(m));
        base = __shfl(base, first);
    }
    const size_t pix = (size_t)py * J.width + px;
    if (hit) {
        const int slot =
            base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        RayRec r;
        for (int a = 0; a < 3; ++a) {
            r.pb[a] = R.pb[a];
            r.d[a] = R.d[a];
        }
        r.kb = R.kb;
        r.ke = R.ke;
        r.t_first = R.t_first;
        r.pixel = (int)pix;
        rays[slot] = r;
    } else if (in_image) {
        reinterpret_cast<float4*>(J.out)[pix] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (J.out_samples) J.out_samples[pix] = 0;
        if (J.out_depth) J.out_depth[pix] = __builtin_inff();
    }
}

template <int INTERP, int G, int SIGK, bool PS>
__device__ __forceinline__ bool pool_row(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R, int lane,
                                         int k0, RayAccum& acc) {
    if constexpr (SIGK >= 0) {
        return lanes_row<INTERP, G, SIGK, PS>(J, s_tf, R, lane, k0, acc);
    } else {
        switch (J.sig) {
        case SIG_F32x1: return lanes_row<INTERP, G, SIG_F32x1, PS>(J, s_tf, R, lane, k0, acc);
        case SIG_PIC3_F32: return lanes_row<INTERP, G, SIG_PIC3_F32, PS>(J, s_tf, R, lane, k0, acc);
        case SIG_PIC3_F16: return lanes_row<INTERP, G, SIG_PIC3_F16, PS>(J, s_tf, R, lane, k0, acc);
        case SIG_PIC3_BF16: return lanes_row<INTERP, G, SIG_PIC3_BF16, PS>(J, s_tf, R, lane, k0, acc);
        case SIG_IL3: return lanes_row<INTERP, G, SIG_IL3, PS>(J, s_tf, R, lane, k0, acc);
        case SIG_IL3P: return lanes_row<INTERP, G, SIG_IL3P, PS>(J, s_tf, R, lane, k0, acc);
        default: return lanes_row<INTERP, G, SIG_GENERIC, PS>(J, s_tf, R, lane, k0, acc);
        }
    }
}

template <int G, int W, int SIGK>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1, 8)))
void raycast_pool_kernel(const DevJob* __restrict__ jobs, const float4* __restrict__ tf_pool,
                         const RayRec* __restrict__ rays, int* __restrict__ counters) {
    extern __shared__ float4 s_tf[];
    const DevJob& J = jobs[0];
    {
        const int n = J.n_src * kTfLds;
        for (int i = (int)threadIdx.x; i < n; i += kBlockThreads)
            s_tf[i] = tf_pool[(size_t)J.src[i / kTfLds].tf_slot * kTfRows + 2 * min(i % kTfLds, kTfEntries - 1)];
        __syncthreads();
    }
    const int n_rays = __builtin_amdgcn_readfirstlane(counters[0]);   // the setup kernel's count
    const int lane = (int)(threadIdx.x & 63);
    const int leader = lane & ~(G - 1);
    constexpr int kChunk = 2 * (64 / G);                                 // rays taken per atomic
    int q_next = 0, q_end = 0;                                           // the wave's local queue
    bool exhausted = false, live = false;
    RaySetup R;
    int pixel = 0, k0 = 0;
    RayAccum acc = {0.f, 0.f, 0.f, 0.f, 0};
    for (;;) {
        // hand queued rays to the idle groups, in lane order
        unsigned long long idle = __ballot(!live && lane == leader);
        while (idle && !exhausted) {
            if (q_next >= q_end) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&counters[1], kChunk);
                base = __shfl(base, 0);
                if (base >= n_rays) {
                    exhausted = true;
                    break;
                }
                q_next = base;
                q_end = min(base + kChunk, n_rays);
            }
            const int take = min(__popcll(idle), q_end - q_next);
            const int rank = __popcll(idle & ((1ull << leader) - 1ull));
            if (!live && rank < take) {
                const RayRec& rr = rays[q_next + rank];
                for (int a = 0; a < 3; ++a) {
                    R.pb[a] = rr.pb[a];
                    R.d[a] = rr.d[a];
                }
                R.kb = rr.kb;
                R.ke = rr.ke;
                R.t_first = rr.t_first;
                pixel = rr.pixel;
                k0 = R.kb;
                acc = RayAccum{0.f, 0.f, 0.f, 0.f, 0};
                live = true;
            }
            q_next += take;
            idle = __ballot(!live && lane == leader);
        }
        if (!__ballot(live)) break;
        if (live) {
            const bool done = J.interp ? pool_row<1, G, SIGK, (W > 0)>(J, s_tf, R, lane, k0, acc)
                                       : pool_row<0, G, SIGK, (W > 0)>(J, s_tf, R, lane, k0, acc);
            k0 += G;
            if (done) {
                if (lane == leader) {
                    reinterpret_cast<float4*>(J.out)[pixel] = make_float4(acc.C0, acc.C1, acc.C2, acc.A);
                    if (J.out_samples) J.out_samples[pixel] = acc.n;
                    if (J.out_depth) J.out_depth[pixel] = R.t_first;
                }
                live = false;
            }
        }
    }
}

// Sort-last compositing of partial images: per pixel, order the layers by
// the ray parameter of their first scan point and apply the front-to-back
// operator (C, A) o (C', A') = (C + (1-A) C', A + (1-A) A').
struct CompositeArgs {
    const float4* rgba[kMaxLayers];
    const float* depth[kMaxLayers];
    int n;
    int64_t n_pixels;
    float4* out;
};

// A layer without a scan point at a pixel has depth +inf and colour
// (0,0,0,0); compositing it changes nothing (C + T*0 = C exactly), so a pixel
// reads the colours of its layers with a finite depth only, and a pixel no
// layer reaches (most of the frame) writes transparent black at once.
__global__ void composite_kernel(CompositeArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_pixels;
         i += (int64_t)gridDim.x * blockDim.x) {
        float dep[kMaxLayers];
        int idx[kMaxLayers];
        int live = 0;
        for (int l = 0; l < a.n; ++l) {
            dep[l] = a.depth[l][i];
            idx[l] = l;
            live += dep[l] < __builtin_inff();
        }
        if (live == 0) {
            a.out[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        for (int l = 1; l < a.n; ++l) {          // insertion sort, stable
            const float dv = dep[l];
            const int iv = idx[l];
            int m = l - 1;
            while (m >= 0 && dep[m] > dv) {
                dep[m + 1] = dep[m];
                idx[m + 1] = idx[m];
                --m;
            }
            dep[m + 1] = dv;
            idx[m + 1] = iv;
        }
        float Cr = 0.f, Cg = 0.f, Cb = 0.f, A = 0.f;
        for (int l = 0; l < live; ++l) {         // the finite depths sort first
            const float4 c = a.rgba[idx[l]][i];
            const float T = 1.f - A;
            Cr = fmaf(T, c.x, Cr);
            Cg = fmaf(T, c.y, Cg);
            Cb = fmaf(T, c.z, Cb);
            A = fmaf(T, c.w, A);
        }
        a.out[i] = make_float4(Cr, Cg, Cb, A);
    }
}

// Frame encode: premultiplied RGBA32F over an opaque background, quantized
// to 8 bits per channel, q = floor(clamp(v, 0, 1) * 255 + 1/2) with NaN -> 0.
// Every operation is a separately rounded FP32 operation (no contraction), so
// the integer codes are a fixed function of the input bits.
struct EncodeArgs {
    const float4* in;
    uchar4* out;
    int64_t n_pixels;
    float bg[3];
    int has_bg;
};

__device__ __forceinline__ unsigned char quantize8(float v) {
#pragma clang fp contract(off)
    const float c = v > 0.f ? fminf(v, 1.f) : 0.f;    // NaN -> 0
    return (unsigned char)(int)floorf(c * 255.f + 0.5f);
}

__global__ void encode_rgba8_kernel(EncodeArgs a) {
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_pixels;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float4 c = a.in[i];
        uchar4 q;
        if (a.has_bg) {
            const float t = 1.f - c.w;
            q.x = quantize8(c.x + t * a.bg[0]);
            q.y = quantize8(c.y + t * a.bg[1]);
            q.z = quantize8(c.z + t * a.bg[2]);
            q.w = 255;
        } else {
            q.x = quantize8(c.x);
            q.y = quantize8(c.y);
            q.z = quantize8(c.z);
            q.w = quantize8(c.w);
        }
        a.out[i] = q;
    }
}

// Derived volume: every voxel's chain output per source, computed once with
// the same fetch and chain code as the ray loop (so the values are the ones
// the loop would compute at that voxel, bit for bit).  A thread takes 4 voxels
// with their loads in flight together: one (x, y) in 4 consecutive z-slices
// (x-fastest layout), or, in the paired layout, both y parities of one stored
// y pair at one x and one z parity in 2 consecutive stored z pairs (its two
// records of a pair are adjacent; lanes alternate the z parity, then step x).
// A wave's stores are one contiguous run (x-fastest) or 64 adjacent record
// pairs, and its reads of a source cover whole runs of 64 or 2 x 32 x.
// SIG > 0: the sources have that signature's compile-time kinds; SIG = 0: any
// sources.
template <int SIG, bool PAIRED>
__device__ __forceinline__ void derive_voxels(const DeriveArgs& a, int xi, int slot, int yi, int zi0, int nz) {
    constexpr int kZ = 4;
    const int ex = a.ext[0], ey = a.ext[1];
    const int x = xi - a.g;
    int vy[kZ], vz[kZ];                        // volume indices of the 4 voxels
    int64_t rec[kZ];                           // their records (float index / n)
    bool need[kZ];
#pragma unroll
    for (int j = 0; j < kZ; ++j) {
        if (PAIRED) {
            // slot: the z parity; j: y parity (j & 1) in stored z pair zi0 + (j >> 1)
            const int zp = zi0 + (j >> 1);
            vy[j] = 2 * yi + (j & 1) - a.gp;
            vz[j] = 2 * zp + slot - a.gp;
            need[j] = (j >> 1) < nz && vy[j] >= -a.g && vy[j] < ey - a.g && vz[j] >= -a.g && vz[j] < a.ext[2] - a.g;
            rec[j] = (((int64_t)zp * a.ny2 + yi) * ex + xi) * 4 + 2 * slot + (j & 1);
        } else {
            vy[j] = yi - a.g;
            vz[j] = zi0 + j - a.g;
            need[j] = j < nz;
            rec[j] = ((int64_t)(zi0 + j) * ey + yi) * ex + xi;
        }
    }
    // The clip test: this latency-bound pass waits on each wave's chain of
    // dependent scalar reads before its loads, so planes are outermost (each read
    // once for the 4 voxels), not one read per voxel and plane.
    if (a.n_sets > 0) {
        // a kept scan point reads voxel centres less than one voxel away per axis
        // (1.5 for the iso-surface gradient), i.e. within 1.5 sqrt(3) < 3 of it
        // along any unit normal
        bool any[kZ] = {false, false, false, false};
        auto test = [&](const float* pl, bool use, bool (&inside)[kZ]) {
            const float n0 = pl[0], n1 = pl[1], n2 = pl[2], n3 = pl[3];
            const float base = n0 * (a.org[0] + x + 0.5f);
#pragma unroll
            for (int j = 0; j < kZ; ++j)
                inside[j] = inside[j] &&
                            (!use || base + n1 * (a.org[1] + vy[j] + 0.5f) + n2 * (a.org[2] + vz[j] + 0.5f) + n3 >= -3.f);
        };
        for (int k = 0; k < a.n_sets; ++k) {
            bool inside[kZ] = {true, true, true, true};
            const int np = a.n_planes[k];
            // the first two planes of a set are read whether used or not (the arrays
            // hold kMaxClip planes), so their loads go out together with the count
            test(a.planes[k][0], np > 0, inside);
            test(a.planes[k][1], np > 1, inside);
            for (int p = 2; p < np; ++p) test(a.planes[k][p], true, inside);
#pragma unroll
            for (int j = 0; j < kZ; ++j) any[j] = any[j] || inside[j];
        }
#pragma unroll
        for (int j = 0; j < kZ; ++j) need[j] = need[j] && any[j];
    }
    int first = -1;
#pragma unroll
    for (int j = kZ - 1; j >= 0; --j)
        if (need[j]) first = j;
    if (first < 0) return;
    // a voxel that is not needed reads the first needed one's address (harmless, never stored)
    int ry[kZ], rz[kZ];
#pragma unroll
    for (int j = 0; j < kZ; ++j) {
        ry[j] = need[j] ? vy[j] : vy[first];
        rz[j] = need[j] ? vz[j] : vz[first];
    }
    // a source without guard layers never has them read: its guard cells hold the border values
    auto offset = [&](const DevSource& S, int y, int z) {
        const int qx = S.guard < 1 ? clampi(x, 0, ex - 2 * a.g - 1) : x;
        const int qy = S.guard < 1 ? clampi(y, 0, ey - 2 * a.g - 1) : y;
        const int qz = S.guard < 1 ? clampi(z, 0, a.ext[2] - 2 * a.g - 1) : z;
        return qx * S.stride[0] + qy * S.stride[1] + qz * S.stride[2];
    };
    auto store = [&](int j, float o0, float o1, float o2, float o3) {
        float* d = a.dst + rec[j] * a.n;
        switch (a.n) {
        case 4: *reinterpret_cast<float4*>(d) = make_float4(o0, o1, o2, o3); break;
        case 3: d[0] = o0; d[1] = o1; d[2] = o2; break;
        case 2: d[0] = o0; d[1] = o1; break;
        default: d[0] = o0; break;
        }
    };
    if constexpr (SIG == SIG_GENERIC) {
        // one voxel at a time (any sources)
#pragma unroll
        for (int j = 0; j < kZ; ++j) {
            if (!need[j]) continue;
            float v[kMaxDerived][1][4];
#pragma unroll
            for (int s = 0; s < kMaxDerived; ++s) {
                if (s < a.n) {
                    const int off[1] = {offset(a.src[s], ry[j], rz[j])};
                    fetch<1>(a.src[s], off, v[s]);
                }
            }
            float o[kMaxDerived] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < kMaxDerived; ++s) {
                if (s < a.n) {
                    float r[1];
                    run_chain<1>(a.src[s], v[s], r);
                    o[s] = r[0];
                }
            }
            store(j, o[0], o[1], o[2], o[3]);
        }
    } else {
        float out[kZ][kMaxDerived];
        constexpr int K0 = SigKinds<SIG>::k0, K1 = SigKinds<SIG>::k1, K2 = SigKinds<SIG>::k2;
        float v0[kZ][4], v1[kZ][4], v2[kZ][4];
        // every load of the 4 voxels first
#pragma unroll
        for (int j = 0; j < kZ; ++j) {
            float t[1][4];
            const int o0[1] = {offset(a.src[0], ry[j], rz[j])};
            fetch_kind<K0, 1>(a.src[0], o0, t);
            for (int c = 0; c < 4; ++c) v0[j][c] = t[0][c];
            if constexpr (K1 != K_NONE) {
                const int o1[1] = {offset(a.src[1], ry[j], rz[j])};
                fetch_kind<K1, 1>(a.src[1], o1, t);
                for (int c = 0; c < 4; ++c) v1[j][c] = t[0][c];
            }
            if constexpr (K2 != K_NONE) {
                const int o2[1] = {offset(a.src[2], ry[j], rz[j])};
                fetch_kind<K2, 1>(a.src[2], o2, t);
                for (int c = 0; c < 4; ++c) v2[j][c] = t[0][c];
            }
        }
#pragma unroll
        for (int j = 0; j < kZ; ++j) {
            float t[1][4], r[1];
            for (int c = 0; c < 4; ++c) t[0][c] = v0[j][c];
            run_chain<1, KindOf<K0>::dim>(a.src[0], t, r);
            out[j][0] = r[0];
            out[j][1] = out[j][2] = out[j][3] = 0.f;
            if constexpr (K1 != K_NONE) {
                for (int c = 0; c < 4; ++c) t[0][c] = v1[j][c];
                run_chain<1, KindOf<K1>::dim>(a.src[1], t, r);
                out[j][1] = r[0];
            }
            if constexpr (K2 != K_NONE) {
                for (int c = 0; c < 4; ++c) t[0][c] = v2[j][c];
                run_chain<1, KindOf<K2>::dim>(a.src[2], t, r);
                out[j][2] = r[0];
            }
        }
        // one contiguous store per voxel
#pragma unroll
        for (int j = 0; j < kZ; ++j)
            if (need[j]) store(j, out[j][0], out[j][1], out[j][2], out[j][3]);
    }
}

// Blocks of 256 threads cover consecutive threads of consecutive rows (y, or
// stored y pairs of 2 ex threads) of one slab (4 z-slices, or 2 stored z
// pairs); grid z strides over the slabs.  Eight waves per SIMD for the paired
// signature-specialized variants: left to itself the compiler keeps the
// arguments in up to 106 scalar registers, which leaves room for seven, and
// this latency-bound pass runs faster with the eighth wave's loads in flight
// (the other variants would spill to scratch under that bound: no bound).
template <int SIG, bool PAIRED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PAIRED && SIG != SIG_GENERIC ? 8 : 1, 8)))
void derive_kernel(DeriveArgs a) {
    const int ex = a.ext[0];
    const int row = PAIRED ? 2 * ex : ex;
    const int rows = PAIRED ? a.ny2 : a.ext[1];
    const int idx = (int)(blockIdx.x * 256 + threadIdx.x);
    if (idx >= row * rows) return;
    const int yi = idx / row;
    const int r = idx - yi * row;
    const int xi = PAIRED ? r >> 1 : r, slot = PAIRED ? r & 1 : 0;
    const int nzs = PAIRED ? a.nz2 : a.ext[2], per = PAIRED ? 2 : 4;
    for (int zi0 = per * (int)blockIdx.z; zi0 < nzs; zi0 += per * (int)gridDim.z)
        derive_voxels<SIG, PAIRED>(a, xi, slot, yi, zi0, min(per, nzs - zi0));
}

// Ray setup of every pixel of each job's screen rectangle, one lane per ray,
// into the job's ray records (kb = ke = 0: no scan point); the ray-casting
// kernel then reads a record instead of repeating the FP64 setup on every
// lane of a ray's group.
__device__ __forceinline__ void ray_setup_dense(const DevJob& J, int block, int n_blocks) {
    const int rw = J.cull[2] - J.cull[0] + 1, rh = J.cull[3] - J.cull[1] + 1;
    if (rw <= 0 || rh <= 0) return;
    RayRec* rays = static_cast<RayRec*>(J.rays);
    for (int i = block * 256 + (int)threadIdx.x; i < rw * rh; i += n_blocks * 256) {
        const int ry = i / rw, rx = i - ry * rw;
        const int px = J.cull[0] + rx, py = J.cull[1] + ry;
        RaySetup R;
        RayRec r;
        if (setup_ray(J, px, py, R)) {
            for (int a = 0; a < 3; ++a) {
                r.pb[a] = R.pb[a];
                r.d[a] = R.d[a];
            }
            r.kb = R.kb;
            r.ke = R.ke;
            r.t_first = R.t_first;
        } else {
            for (int a = 0; a < 3; ++a) r.pb[a] = r.d[a] = 0.f;
            r.kb = r.ke = 0;
            r.t_first = 0.f;
        }
        r.pixel = py * J.width + px;
        rays[i] = r;
    }
}

// Clear the output of every pixel outside its job's screen rectangle (no ray
// there can meet the box): transparent black, 0 samples, depth +inf.
__device__ __forceinline__ void fill_outside(const DevJob& J, int block, int n_blocks) {
    const int n = J.width * J.height;
    for (int i = block * 256 + (int)threadIdx.x; i < n; i += n_blocks * 256) {
        const int py = i / J.width, px = i - py * J.width;
        if (px >= J.cull[0] && px <= J.cull[2] && py >= J.cull[1] && py <= J.cull[3]) continue;
        reinterpret_cast<float4*>(J.out)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (J.out_samples) J.out_samples[i] = 0;
        if (J.out_depth) J.out_depth[i] = __builtin_inff();
    }
}

__global__ __launch_bounds__(256) void fill_outside_kernel(const DevJob* __restrict__ jobs) {
    fill_outside(jobs[blockIdx.y], (int)blockIdx.x, (int)gridDim.x);
}

// The fill and the ray setup touch different memory: one launch runs both,
// workgroups [0, nb) filling and [nb, 2 nb) setting up rays.
__global__ __launch_bounds__(256) void prepass_kernel(const DevJob* __restrict__ jobs, int nb) {
    const DevJob& J = jobs[blockIdx.y];
    const int b = (int)blockIdx.x;
    if (b < nb)
        fill_outside(J, b, nb);
    else
        ray_setup_dense(J, b - nb, nb);
}

// One job: the fill and ray setup as above, reading the job block from the
// kernel arguments, and the block stored to device memory for the
// ray-casting launch that follows (no separate host-to-device copy).
__global__ __launch_bounds__(256) void prepass_one_kernel(const DevJob job, DevJob* __restrict__ dst, int nb,
                                                          int dense) {
    const int b = (int)blockIdx.x;
    if (b == 0) {
        const uint32_t* s = reinterpret_cast<const uint32_t*>(&job);
        uint32_t* d = reinterpret_cast<uint32_t*>(dst);
        for (int i = (int)threadIdx.x; i < (int)(sizeof(DevJob) / 4); i += 256) d[i] = s[i];
    }
    if (b < nb)
        fill_outside(job, b, nb);
    else if (dense)
        ray_setup_dense(job, b - nb, nb);
}

__global__ void reset_counter_kernel(int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Copy a strided field (guard layers included) into a packed buffer of the
// same storage type.  One thread per voxel.
struct CopyArgs {
    const unsigned char* src[4];
    int64_t src_stride[3];
    unsigned char* dst;
    int64_t dst_stride[3];
    int esize, f_dim;
    int lo[3], ext[3];
};

__global__ __launch_bounds__(256) void strided_copy_kernel(CopyArgs a) {
    const int xi = (int)(blockIdx.x * 64 + threadIdx.x);
    const int yi = (int)(blockIdx.y * 4 + threadIdx.y);
    if (xi >= a.ext[0] || yi >= a.ext[1]) return;
    for (int zi = (int)blockIdx.z; zi < a.ext[2]; zi += (int)gridDim.z) {
        const int x = xi + a.lo[0];
        const int y = yi + a.lo[1];
        const int z = zi + a.lo[2];
        for (int c = 0; c < a.f_dim; ++c) {
            const unsigned char* s = a.src[c] + x * a.src_stride[0] + y * a.src_stride[1] + z * a.src_stride[2];
            unsigned char* d = a.dst + x * a.dst_stride[0] + y * a.dst_stride[1] + z * a.dst_stride[2] +
                               (int64_t)c * a.esize;
            if (a.esize == 4) *reinterpret_cast<uint32_t*>(d) = *reinterpret_cast<const uint32_t*>(s);
            else *reinterpret_cast<uint16_t*>(d) = *reinterpret_cast<const uint16_t*>(s);
        }
    }
}

}  // namespace

using KernelFn = void (*)(const DevJob*, const float4*, int*, int, int, int);

template <int SIGK>
KernelFn pick_specialized(int unroll, int lanes, int hint) {
    if (unroll >= 2) return raycast_kernel<2, 1, 0, SIGK>;
    switch (lanes) {
    case 64: return raycast_kernel<1, 64, 0, SIGK>;
    case 32: return raycast_kernel<1, 32, 0, SIGK>;
    case 16: return hint ? raycast_kernel<1, 16, 4, SIGK> : raycast_kernel<1, 16, 0, SIGK>;
    case 8: return hint ? raycast_kernel<1, 8, 4, SIGK> : raycast_kernel<1, 8, 0, SIGK>;
    case 4: return hint ? raycast_kernel<1, 4, 4, SIGK> : raycast_kernel<1, 4, 0, SIGK>;
    case 2: return raycast_kernel<1, 2, 0, SIGK>;
    default: return hint ? raycast_kernel<1, 1, 4, SIGK> : raycast_kernel<1, 1, 0, SIGK>;
    }
}

KernelFn pick_kernel(int mode, int sig, int unroll, int lanes, int hint) {
    if (mode == 1) {
        // iso-surface jobs: sig -3 when every source is plain (packed FP32 scalars without
        // functors, guard layers), else the run-time source handling
        if (sig == -3) return lanes >= 8 ? raycast_kernel<1, 8, 0, -3> : raycast_kernel<1, 1, 0, -3>;
        return lanes >= 8 ? raycast_kernel<1, 8, 0, -2> : raycast_kernel<1, 1, 0, -2>;
    }
    switch (sig) {
    case SIG_F32x1: return pick_specialized<SIG_F32x1>(unroll, lanes, hint);
    case SIG_PIC3_F32: return pick_specialized<SIG_PIC3_F32>(unroll, lanes, hint);
    case SIG_PIC3_F16: return pick_specialized<SIG_PIC3_F16>(unroll, lanes, hint);
    case SIG_PIC3_BF16: return pick_specialized<SIG_PIC3_BF16>(unroll, lanes, hint);
    case SIG_IL3: return pick_specialized<SIG_IL3>(unroll, lanes, hint);
    case SIG_IL3P: return pick_specialized<SIG_IL3P>(unroll, lanes, hint);
    default:
        break;
    }
    // mixed or generic signatures: the dispatching kernels (one lane-count each)
    switch (lanes) {
    case 64: return raycast_kernel<1, 64, 0, -1>;
    case 32: return raycast_kernel<1, 32, 0, -1>;
    case 16: return raycast_kernel<1, 16, 0, -1>;
    case 8: return raycast_kernel<1, 8, 0, -1>;
    case 4: return raycast_kernel<1, 4, 0, -1>;
    case 2: return raycast_kernel<1, 2, 0, -1>;
    default: return raycast_kernel<1, 1, 0, -1>;
    }
}

int launch_prepass(const LaunchArgs& a, void* stream) {
    // pixels outside the jobs' screen rectangles, then (optionally) the rays inside them
    if (a.dense_setup)
        hipLaunchKernelGGL(prepass_kernel, dim3(2 * a.fill_blocks, (unsigned)a.n_jobs), dim3(256), 0,
                           (hipStream_t)stream, a.jobs, (int)a.fill_blocks);
    else
        hipLaunchKernelGGL(fill_outside_kernel, dim3(a.fill_blocks, (unsigned)a.n_jobs), dim3(256), 0,
                           (hipStream_t)stream, a.jobs);
    return hipGetLastError();
}

int launch_prepass_one(const DevJob& job, DevJob* dst, unsigned fill_blocks, int dense, void* stream) {
    static_assert(sizeof(DevJob) % 4 == 0 && sizeof(DevJob) + 16 <= 4096, "the job block is a kernel argument");
    hipLaunchKernelGGL(prepass_one_kernel, dim3((dense ? 2 : 1) * fill_blocks), dim3(256), 0, (hipStream_t)stream,
                       job, dst, (int)fill_blocks, dense);
    return hipGetLastError();
}

int launch_raycast(const LaunchArgs& a, void* stream) {
    // dynamic LDS: one staged table (kTfLds RGBA32F values) per active source of the widest job
    const size_t lds = (size_t)(a.max_src > 0 ? a.max_src : 1) * kTfLds * sizeof(float4);
    const unsigned blocks = a.persistent ? (unsigned)a.grid : (unsigned)a.total_tiles;
    if (blocks == 0) return hipGetLastError();
    const KernelFn kernel = pick_kernel(a.mode, a.sig, a.unroll, a.lanes, a.waves_hint);
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kBlockThreads), lds, (hipStream_t)stream, a.jobs,
                       reinterpret_cast<const float4*>(a.tf_pool), a.cursor, a.n_jobs, a.total_tiles, a.persistent);
    return hipGetLastError();
}

using PoolFn = void (*)(const DevJob*, const float4*, const RayRec*, int*);

template <int SIGK>
PoolFn pick_pool_specialized(int lanes, int hint) {
    switch (lanes) {
    case 16: return hint ? raycast_pool_kernel<16, 4, SIGK> : raycast_pool_kernel<16, 0, SIGK>;
    case 8: return hint ? raycast_pool_kernel<8, 4, SIGK> : raycast_pool_kernel<8, 0, SIGK>;
    case 4: return hint ? raycast_pool_kernel<4, 4, SIGK> : raycast_pool_kernel<4, 0, SIGK>;
    default: return raycast_pool_kernel<2, 0, SIGK>;
    }
}

PoolFn pick_pool_kernel(int sig, int lanes, int hint) {
    switch (sig) {
    case SIG_F32x1: return pick_pool_specialized<SIG_F32x1>(lanes, hint);
    case SIG_PIC3_F32: return pick_pool_specialized<SIG_PIC3_F32>(lanes, hint);
    case SIG_PIC3_F16: return pick_pool_specialized<SIG_PIC3_F16>(lanes, hint);
    case SIG_PIC3_BF16: return pick_pool_specialized<SIG_PIC3_BF16>(lanes, hint);
    case SIG_IL3: return pick_pool_specialized<SIG_IL3>(lanes, hint);
    case SIG_IL3P: return pick_pool_specialized<SIG_IL3P>(lanes, hint);
    default: break;
    }
    switch (lanes) {
    case 16: return raycast_pool_kernel<16, 0, -1>;
    case 8: return raycast_pool_kernel<8, 0, -1>;
    case 4: return raycast_pool_kernel<4, 0, -1>;
    default: return raycast_pool_kernel<2, 0, -1>;
    }
}

int launch_raycast_pooled(const DevJob* job_dev, int width, int height, const float* tf_pool, int max_src, int sig,
                          int lanes, int hint, void* rays, int* counters, int n_cu, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, counters, 2);
    const dim3 sgrid((unsigned)((width + 15) / 16), (unsigned)((height + 15) / 16));
    hipLaunchKernelGGL(ray_setup_kernel, sgrid, dim3(256), 0, st, job_dev, static_cast<RayRec*>(rays), counters);
    const size_t lds = (size_t)(max_src > 0 ? max_src : 1) * kTfLds * sizeof(float4);
    const PoolFn k = pick_pool_kernel(sig, lanes, hint);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlockThreads, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    hipLaunchKernelGGL(k, dim3((unsigned)(n_cu * per_cu)), dim3(kBlockThreads), lds, st, job_dev,
                       reinterpret_cast<const float4*>(tf_pool), static_cast<const RayRec*>(rays), counters);
    return hipGetLastError();
}

size_t ray_record_bytes() { return sizeof(RayRec); }

int launch_reset_counter(int* counter, void* stream) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, counter, 1);
    return hipGetLastError();
}

int launch_strided_copy(const void* const* src_comp, const int64_t* src_stride, void* dst,
                        const int64_t* dst_stride, int esize, int f_dim, const int32_t lo[3],
                        const int32_t ext[3], void* stream) {
    CopyArgs a;
    for (int c = 0; c < 4; ++c) a.src[c] = c < f_dim ? static_cast<const unsigned char*>(src_comp[c]) : nullptr;
    for (int k = 0; k < 3; ++k) {
        a.src_stride[k] = src_stride[k];
        a.dst_stride[k] = dst_stride[k];
        a.lo[k] = lo[k];
        a.ext[k] = ext[k];
    }
    a.dst = static_cast<unsigned char*>(dst);
    a.esize = esize;
    a.f_dim = f_dim;
    if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ext[0] + 63) / 64), (unsigned)((ext[1] + 3) / 4), (unsigned)std::min(ext[2], 65535));
    hipLaunchKernelGGL(strided_copy_kernel, grid, dim3(64, 4), 0, (hipStream_t)stream, a);
    return hipGetLastError();
}

int launch_composite(const float* const* rgba, const float* const* depth, int n_layers, int64_t n_pixels, float* out,
                     void* stream) {
    CompositeArgs a;
    for (int l = 0; l < kMaxLayers; ++l) {
        a.rgba[l] = l < n_layers ? reinterpret_cast<const float4*>(rgba[l]) : nullptr;
        a.depth[l] = l < n_layers ? depth[l] : nullptr;
    }
    a.n = n_layers;
    a.n_pixels = n_pixels;
    a.out = reinterpret_cast<float4*>(out);
    if (n_pixels <= 0) return hipSuccess;
    const int64_t blocks = (n_pixels + 255) / 256;
    hipLaunchKernelGGL(composite_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                       (hipStream_t)stream, a);
    return hipGetLastError();
}

int launch_encode_rgba8(const float* rgba, int64_t n_pixels, const float* bg, unsigned char* out, void* stream) {
    EncodeArgs a;
    a.in = reinterpret_cast<const float4*>(rgba);
    a.out = reinterpret_cast<uchar4*>(out);
    a.n_pixels = n_pixels;
    a.has_bg = bg != nullptr;
    for (int c = 0; c < 3; ++c) a.bg[c] = bg ? bg[c] : 0.f;
    const int64_t blocks = std::min<int64_t>((n_pixels + 255) / 256, 8192);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(encode_rgba8_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError();
}

template <bool PAIRED>
void (*derive_variant(int sig))(DeriveArgs) {
    switch (sig) {
    case SIG_F32x1: return derive_kernel<SIG_F32x1, PAIRED>;
    case SIG_PIC3_F32: return derive_kernel<SIG_PIC3_F32, PAIRED>;
    case SIG_PIC3_F16: return derive_kernel<SIG_PIC3_F16, PAIRED>;
    case SIG_PIC3_BF16: return derive_kernel<SIG_PIC3_BF16, PAIRED>;
    default: return derive_kernel<SIG_GENERIC, PAIRED>;
    }
}

int launch_derive(const DeriveArgs& a, int sig, void* stream) {
    if (a.ext[0] <= 0 || a.ext[1] <= 0 || a.ext[2] <= 0) return hipSuccess;
    if (a.paired && (a.gp < a.g || (a.gp & 1) || 2 * a.ny2 < a.ext[1] - a.g + a.gp ||
                     2 * a.nz2 < a.ext[2] - a.g + a.gp))
        return hipErrorInvalidValue;
    const int64_t slice = (int64_t)a.ext[0] * (a.paired ? 2 * (int64_t)a.ny2 : a.ext[1]);
    if (slice > (1LL << 30)) return hipErrorInvalidValue;
    const int slabs = a.paired ? (a.nz2 + 1) / 2 : (a.ext[2] + 3) / 4;
    const dim3 grid((unsigned)((slice + 255) / 256), 1, (unsigned)std::min(slabs, 65535));
    void (*k)(DeriveArgs) = a.paired ? derive_variant<true>(sig) : derive_variant<false>(sig);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError();
}

// Scratch of the render entry point that allocates nothing: the ray records of
// its set-up pass.  One copy per device, held until the process ends; every call
// on a device uses that device's copy, so calls that overlap on one device (other
// streams, other contexts) race.  Host code must not pass the array's name to a
// kernel (in host code it is a stand-in, not a device address): it takes the
// address noalloc_scratch() looked up for the device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int noalloc_scratch(int device, void** ptr) {
    static std::mutex lock;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

int raycast_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, raycast_kernel<1, 1, 0, -1>, kBlockThreads,
                                                       3 * kTfLds * sizeof(float4));
}

}  // namespace isaac
