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
// N dates of work inside.  res[i] is component 0 of date i's result.
template <int N>
__device__ __forceinline__ void run_chain(const DevSource& S, float (&v)[N][4], float (&res)[N]) {
    const int n_ops = S.n_ops;
    for (int o = 0; o < n_ops; ++o) {
        const DevOp& op = S.ops[o];
        const int dim = op.dim;
        const float a[4] = {op.arg[0], op.arg[1], op.arg[2], op.arg[3]};
        switch (op.kind) {
        case OP_ADD:
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] + a[c];
            break;
        case OP_MUL:
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] * a[c];
            break;
        case OP_POW:
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = pow_f32(v[i][c], a[c]);
            break;
        case OP_SQRT:
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i)
                        v[i][c] = v[i][c] < 0.f ? __builtin_nanf("") : __builtin_amdgcn_sqrtf(v[i][c]);
            break;
        case OP_SQUARE:
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < dim)
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i][c] = v[i][c] * v[i][c];
            break;
        case OP_LENGTH:
            if (dim == 3) {
#pragma unroll
                for (int i = 0; i < N; ++i)
                    v[i][0] = __builtin_amdgcn_sqrtf(fmaf(v[i][2], v[i][2], fmaf(v[i][1], v[i][1], v[i][0] * v[i][0])));
            } else {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    float s = v[i][0] * v[i][0];
                    if (dim > 1) s = fmaf(v[i][1], v[i][1], s);
                    if (dim > 2) s = fmaf(v[i][2], v[i][2], s);
                    if (dim > 3) s = fmaf(v[i][3], v[i][3], s);
                    v[i][0] = __builtin_amdgcn_sqrtf(s);
                }
            }
            break;
        case OP_SUM:
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float s = v[i][0];
                if (dim > 1) s = s + v[i][1];
                if (dim > 2) s = s + v[i][2];
                if (dim > 3) s = s + v[i][3];
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

// Transfer-table lookup: clamp to [0,1] (NaN -> 0), 255 intervals, linear.
__device__ __forceinline__ float4 classify(const float4* __restrict__ table, float x) {
    float t = (x > 0.f) ? fminf(x, 1.f) : 0.f;
    float u = 255.f * t;
    int j = min((int)u, 254);
    float f = u - (float)j;
    float4 a = table[j];
    float4 b = table[j + 1];
    return make_float4(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y), fmaf(f, b.z - a.z, a.z),
                       fmaf(f, b.w - a.w, a.w));
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// FP64 ray setup.  Returns false if the ray misses the box or keeps no scan
// point; otherwise the kept sample indices are [*kb, *ke) and the FP32 ray is
// p(k) = pb + ((k + 1/2) * step) * d32.
struct RaySetup {
    float pb[3];
    float d[3];
    int kb, ke;
};

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
    // slab test against [0, N]
    double lo = -__builtin_inf(), hi = __builtin_inf();
    for (int a = 0; a < 3; ++a) {
        const double nn = (double)J.dims[a];
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > nn) return false;
            continue;
        }
        const double ta = (0.0 - o[a]) / d[a];
        const double tb = (nn - o[a]) / d[a];
        const double tn = ta < tb ? ta : tb;
        const double tf = ta < tb ? tb : ta;
        if (tn > lo) lo = tn;
        if (tf < hi) hi = tf;
    }
    if (lo < 0.0) lo = 0.0;
    if (!(hi > lo)) return false;
    const double t0 = lo, t1 = hi, step = J.step;
    // number of k >= 0 with t0 + (k + 1/2) step < t1
    double r = (t1 - t0) / step - 0.5;
    int n = r > 0.0 ? (int)fmin(ceil(r), 2147483000.0) : 0;
    while (n > 0 && !(t0 + ((double)(n - 1) + 0.5) * step < t1)) --n;
    while (t0 + ((double)n + 0.5) * step < t1) ++n;
    int kb = 0, ke = n;
    // each plane keeps one interval of k; evaluate the plane at p(k) exactly
    // as written (o + t d, then n.p + d) at the interval ends
    for (int c = 0; c < J.n_clip && kb < ke; ++c) {
        const double* pl = J.clip[c];
        const double nd = pl[0] * d[0] + pl[1] * d[1] + pl[2] * d[2];
        auto keep = [&](int k) {
#pragma clang fp contract(off)
            const double t = t0 + ((double)k + 0.5) * step;
            const double p0 = o[0] + t * d[0], p1 = o[1] + t * d[1], p2 = o[2] + t * d[2];
            return pl[0] * p0 + pl[1] * p1 + pl[2] * p2 + pl[3] >= 0.0;
        };
        const double no = pl[0] * o[0] + pl[1] * o[1] + pl[2] * o[2] + pl[3];
        if (nd == 0.0) {
            if (!keep(kb)) ke = kb;
            continue;
        }
        // crossing parameter and the sample index near it
        const double tc = -no / nd;
        double kc = (tc - t0) / step - 0.5;
        kc = fmin(fmax(kc, (double)kb - 1.0), (double)ke + 1.0);
        int k = (int)ceil(kc);
        if (nd > 0.0) {     // kept for k >= first kept index
            k = clampi(k, kb, ke);
            while (k > kb && keep(k - 1)) --k;
            while (k < ke && !keep(k)) ++k;
            kb = k;
        } else {            // kept for k < first dropped index
            k = clampi(k, kb, ke);
            while (k < ke && keep(k)) ++k;
            while (k > kb && !keep(k - 1)) --k;
            ke = k;
        }
    }
    if (kb >= ke) return false;
    for (int a = 0; a < 3; ++a) {
        R.pb[a] = (float)(o[a] + t0 * d[a]);
        R.d[a] = (float)d[a];
    }
    R.kb = kb;
    R.ke = ke;
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

template <int INTERP>
__device__ __forceinline__ void march(const DevJob& J, const float4* __restrict__ s_tf, const RaySetup& R, float4& out,
                      int& count) {
    const float step = (float)J.step;
    const float ert = J.ert;
    const int n_src = J.n_src;
    const int dims[3] = {J.dims[0], J.dims[1], J.dims[2]};
    float Cr = 0.f, Cg = 0.f, Cb = 0.f, A = 0.f;
    int n = 0;
    for (int k = R.kb; k < R.ke; ++k) {
        const float tk = ((float)k + 0.5f) * step;
        const float p[3] = {fmaf(tk, R.d[0], R.pb[0]), fmaf(tk, R.d[1], R.pb[1]), fmaf(tk, R.d[2], R.pb[2])};
        float S = 0.f, Er = 0.f, Eg = 0.f, Eb = 0.f;
        for (int s = 0; s < n_src; ++s) {
            const DevSource& src = J.src[s];
            const float x = sample_source<INTERP>(src, dims, p);
            const float4 c = classify(s_tf + s * kTfEntries, x);
            const float wa = src.weight * c.w;
            S += wa;
            Er = fmaf(wa, c.x, Er);
            Eg = fmaf(wa, c.y, Eg);
            Eb = fmaf(wa, c.z, Eb);
        }
        if (S > 1.f) {
            const float inv = 1.f / S;
            Er *= inv;
            Eg *= inv;
            Eb *= inv;
            S = 1.f;
        }
        const float T = 1.f - A;
        Cr = fmaf(T, Er, Cr);
        Cg = fmaf(T, Eg, Cg);
        Cb = fmaf(T, Eb, Cb);
        A = fmaf(T, S, A);
        ++n;
        if (A >= ert) break;
    }
    out = make_float4(Cr, Cg, Cb, A);
    count = n;
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

__device__ __forceinline__ void render_tile(const DevJob& J, int t, const float4* __restrict__ s_tf) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ww = J.wave_w, wh = 64 / ww;
    const int gx = J.waves_x, gy = 4 / gx;
    const int tx = t % J.tiles_x, ty = t / J.tiles_x;
    const int px = tx * (ww * gx) + (wave % gx) * ww + lane % ww;
    const int py = ty * (wh * gy) + (wave / gx) * wh + lane / ww;
    if (px >= J.width || py >= J.height) return;
    RaySetup R;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    int count = 0;
    if (setup_ray(J, px, py, R)) {
        if (J.interp) march<1>(J, s_tf, R, c, count);
        else march<0>(J, s_tf, R, c, count);
    }
    const size_t pix = (size_t)py * J.width + px;
    reinterpret_cast<float4*>(J.out)[pix] = c;
    if (J.out_samples) J.out_samples[pix] = count;
}

__global__ __launch_bounds__(kBlockThreads) void raycast_kernel(const DevJob* __restrict__ jobs,
                                                                 const float4* __restrict__ tf_pool,
                                                                 int* __restrict__ cursor, int n_jobs,
                                                                 int total_tiles, int persistent) {
    extern __shared__ float4 s_tf[];
    __shared__ int s_tile;
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
        if (job != cur_job) {
            __syncthreads();
            const int n = J.n_src * kTfEntries;
            for (int i = threadIdx.x; i < n; i += kBlockThreads) {
                const int s = i / kTfEntries, e = i % kTfEntries;
                s_tf[i] = tf_pool[(size_t)J.src[s].tf_slot * kTfEntries + e];
            }
            __syncthreads();
            cur_job = job;
        }
        render_tile(J, tile - J.tile_begin, s_tf);
    }
}

__global__ void reset_counter_kernel(int* c) {
    if (threadIdx.x == 0) c[0] = 0;
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

__global__ void strided_copy_kernel(CopyArgs a) {
    const int64_t n = (int64_t)a.ext[0] * a.ext[1] * a.ext[2];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.ext[0]) + a.lo[0];
        const int y = (int)((i / a.ext[0]) % a.ext[1]) + a.lo[1];
        const int z = (int)(i / ((int64_t)a.ext[0] * a.ext[1])) + a.lo[2];
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

int launch_raycast(const LaunchArgs& a, void* stream) {
    // dynamic LDS: one 256-entry RGBA32F table per active source of the widest job
    const size_t lds = (size_t)(a.max_src > 0 ? a.max_src : 1) * kTfEntries * sizeof(float4);
    const unsigned blocks = a.persistent ? (unsigned)a.grid : (unsigned)a.total_tiles;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(raycast_kernel, dim3(blocks), dim3(kBlockThreads), lds, (hipStream_t)stream, a.jobs,
                       reinterpret_cast<const float4*>(a.tf_pool), a.cursor, a.n_jobs, a.total_tiles, a.persistent);
    return hipGetLastError();
}

int launch_reset_counter(int* counter, void* stream) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, counter);
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
    const int64_t n = (int64_t)ext[0] * ext[1] * ext[2];
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(strided_copy_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                       (hipStream_t)stream, a);
    return hipGetLastError();
}

int raycast_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, raycast_kernel, kBlockThreads,
                                                       3 * kTfEntries * sizeof(float4));
}

}  // namespace isaac
