/*
 * FP64 single-threaded CPU oracle of the ISAAC volume ray caster.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU baseline of the benchmark, never by the GPU library.  Plain C, no
 * blocking, no reordering: every step is written in the order the method
 * takes it, one pixel, one scan point, one source at a time.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 *
 * Pins: closed forms (constant slab, linear ramp), the paper's two worked
 * functor examples, a brute-force per-sample loop on tiny grids, ray/box
 * geometry special cases and the early-termination bound (tests/).
 */
#include "isaac_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAX_OPS 8
#define MAX_SRC 16
#define TF_SIZE 256
#define ORACLE_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* error reporting                                                      */
/* ------------------------------------------------------------------ */
static int fail(char* err, int errlen, const char* fmt, ...) {
    if (err && errlen > 0) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(err, (size_t)errlen, fmt, ap);
        va_end(ap);
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* functor chains (Sec. 3.3, Tab. "functors")                           */
/*   add(v), mul(v), pow(v): componentwise, R^n -> R^n; a single         */
/*       argument applies to every component ("add(1)" adds (1,1,1));   */
/*   length: R^n -> R, Euclidean length;                                 */
/*   sum:    R^n -> R, sum of the components;                            */
/*   an unreduced vector yields its first component.                     */
/* ------------------------------------------------------------------ */
enum { OP_ADD, OP_MUL, OP_POW, OP_LENGTH, OP_SUM };

typedef struct {
    int kind;
    int nargs;
    double arg[4];
} functor;

typedef struct {
    int n_ops;
    int in_dim;
    functor op[MAX_OPS];
} chain;

static const char* skip_ws(const char* s) {
    while (*s == ' ' || *s == '\t' || *s == '\n' || *s == '\r') s++;
    return s;
}

static int parse_chain(const char* text, int f_dim, chain* out, char* err, int errlen) {
    memset(out, 0, sizeof(*out));
    out->in_dim = f_dim;
    if (f_dim < 1 || f_dim > 4) return fail(err, errlen, "f_dim %d outside 1..4", f_dim);
    if (!text) return 0;
    const char* s = skip_ws(text);
    if (*s == 0) return 0;
    int dim = f_dim;
    for (;;) {
        char name[16];
        int len = 0;
        while ((*s >= 'a' && *s <= 'z') && len < 15) name[len++] = *s++;
        name[len] = 0;
        if (len == 0) return fail(err, errlen, "expected a functor name at '%s'", s);
        functor f;
        memset(&f, 0, sizeof(f));
        int takes_args;
        if (strcmp(name, "add") == 0) { f.kind = OP_ADD; takes_args = 1; }
        else if (strcmp(name, "mul") == 0) { f.kind = OP_MUL; takes_args = 1; }
        else if (strcmp(name, "pow") == 0) { f.kind = OP_POW; takes_args = 1; }
        else if (strcmp(name, "length") == 0) { f.kind = OP_LENGTH; takes_args = 0; }
        else if (strcmp(name, "sum") == 0) { f.kind = OP_SUM; takes_args = 0; }
        else return fail(err, errlen, "unknown functor '%s'", name);
        s = skip_ws(s);
        if (*s == '(') {
            s = skip_ws(s + 1);
            if (*s == ')') {
                s++;
            } else {
                for (;;) {
                    char* end;
                    double v = strtod(s, &end);
                    if (end == s) return fail(err, errlen, "expected a number in '%s'", name);
                    if (f.nargs == 4) return fail(err, errlen, "more than 4 arguments to '%s'", name);
                    f.arg[f.nargs++] = v;
                    s = skip_ws(end);
                    if (*s == ',') { s = skip_ws(s + 1); continue; }
                    if (*s == ')') { s++; break; }
                    return fail(err, errlen, "expected ',' or ')' in '%s'", name);
                }
            }
        }
        if (takes_args) {
            if (f.nargs != 1 && f.nargs != dim)
                return fail(err, errlen, "'%s' takes 1 or %d arguments, got %d", name, dim, f.nargs);
        } else if (f.nargs != 0) {
            return fail(err, errlen, "'%s' takes no arguments", name);
        }
        if (out->n_ops == MAX_OPS) return fail(err, errlen, "more than %d functors", MAX_OPS);
        out->op[out->n_ops++] = f;
        if (f.kind == OP_LENGTH || f.kind == OP_SUM) dim = 1;
        s = skip_ws(s);
        if (*s == 0) break;
        if (*s != '|') return fail(err, errlen, "expected '|' at '%s'", s);
        s = skip_ws(s + 1);
    }
    return 0;
}

/* Applies the chain to v[0..f_dim); returns component 0 of the result. */
static double apply_chain(const chain* c, const double* in, int* out_dim) {
    double v[4] = {0, 0, 0, 0};
    int dim = c->in_dim;
    for (int k = 0; k < dim; k++) v[k] = in[k];
    for (int o = 0; o < c->n_ops; o++) {
        const functor* f = &c->op[o];
        switch (f->kind) {
        case OP_ADD:
            for (int k = 0; k < dim; k++) v[k] = v[k] + (f->nargs == 1 ? f->arg[0] : f->arg[k]);
            break;
        case OP_MUL:
            for (int k = 0; k < dim; k++) v[k] = v[k] * (f->nargs == 1 ? f->arg[0] : f->arg[k]);
            break;
        case OP_POW:
            for (int k = 0; k < dim; k++) v[k] = pow(v[k], f->nargs == 1 ? f->arg[0] : f->arg[k]);
            break;
        case OP_LENGTH: {
            double s = 0.0;
            for (int k = 0; k < dim; k++) s += v[k] * v[k];
            v[0] = sqrt(s);
            dim = 1;
            break;
        }
        case OP_SUM: {
            double s = 0.0;
            for (int k = 0; k < dim; k++) s += v[k];
            v[0] = s;
            dim = 1;
            break;
        }
        }
    }
    if (out_dim) *out_dim = dim;
    return v[0];
}

int oracle_chain_eval(const char* text, int f_dim, const double* in, double* out, int* out_dim,
                      char* err, int errlen) {
    chain c;
    if (parse_chain(text, f_dim, &c, err, errlen)) return -1;
    *out = apply_chain(&c, in, out_dim);
    return 0;
}

/* ------------------------------------------------------------------ */
/* transfer function: piecewise linear RGBA over [0,1], tabulated at     */
/* j/255 for j = 0..255, looked up with linear interpolation             */
/* ------------------------------------------------------------------ */
static int check_tf(int n, const double* tf, char* err, int errlen) {
    if (n < 2) return fail(err, errlen, "transfer function needs at least 2 points");
    if (tf[0] != 0.0 || tf[5 * (n - 1)] != 1.0)
        return fail(err, errlen, "transfer function must span [0,1]");
    for (int i = 0; i < n; i++) {
        for (int c = 0; c < 5; c++) {
            double v = tf[5 * i + c];
            if (!(v >= 0.0 && v <= 1.0)) return fail(err, errlen, "transfer function value outside [0,1]");
        }
        if (i > 0 && !(tf[5 * i] > tf[5 * (i - 1)]))
            return fail(err, errlen, "transfer function x not strictly increasing");
    }
    return 0;
}

static void piecewise_linear(int n, const double* tf, double x, double rgba[4]) {
    int i = 0;
    while (i < n - 2 && x > tf[5 * (i + 1)]) i++;
    double x0 = tf[5 * i], x1 = tf[5 * (i + 1)];
    double w = (x - x0) / (x1 - x0);
    for (int c = 0; c < 4; c++) {
        double a = tf[5 * i + 1 + c], b = tf[5 * (i + 1) + 1 + c];
        rgba[c] = a + w * (b - a);
    }
}

int oracle_tf_table(int n, const double* tf, double* table, char* err, int errlen) {
    if (check_tf(n, tf, err, errlen)) return -1;
    for (int j = 0; j < TF_SIZE; j++) piecewise_linear(n, tf, (double)j / 255.0, table + 4 * j);
    return 0;
}

/* classification of the chain output x */
static void classify(const double* table, double x, double rgba[4]) {
    double t = isnan(x) ? 0.0 : (x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x));
    double u = 255.0 * t;
    int j = (int)floor(u);
    if (j > 254) j = 254;
    double f = u - (double)j;
    for (int c = 0; c < 4; c++) rgba[c] = table[4 * j + c] + f * (table[4 * (j + 1) + c] - table[4 * j + c]);
}

/* ------------------------------------------------------------------ */
/* source access through the accessor (pointer + byte strides)          */
/* ------------------------------------------------------------------ */
static double half_to_double(uint16_t h) {
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0) v = ldexp((double)m, -24);                 /* zero or subnormal */
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m | 0x400), e - 25);
    return sign ? -v : v;
}

static double bf16_to_double(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double read_component(const oracle_source* s, int c, int x, int y, int z) {
    const unsigned char* p = s->comp[c] + (int64_t)x * s->stride[0] + (int64_t)y * s->stride[1] +
                             (int64_t)z * s->stride[2];
    if (s->dtype == ORACLE_F32) {
        float f;
        memcpy(&f, p, 4);
        return (double)f;
    }
    uint16_t h;
    memcpy(&h, p, 2);
    return s->dtype == ORACLE_F16 ? half_to_double(h) : bf16_to_double(h);
}

/* ------------------------------------------------------------------ */
/* prepared scene                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    const oracle_scene* sc;
    chain ch[MAX_SRC];
    double table[MAX_SRC][TF_SIZE * 4];
    double fwd[3], right[3], upp[3], h, aspect;
} prepared;

static void cross3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void normalize3(double v[3]) {
    double n = sqrt(dot3(v, v));
    v[0] /= n; v[1] /= n; v[2] /= n;
}

static int prepare(const oracle_scene* sc, prepared* P, char* err, int errlen) {
    P->sc = sc;
    for (int a = 0; a < 3; a++)
        if (sc->dims[a] < 1) return fail(err, errlen, "dims must be positive");
    if (sc->n_src < 0 || sc->n_src > MAX_SRC) return fail(err, errlen, "at most %d sources", MAX_SRC);
    if (!(sc->step > 0.0)) return fail(err, errlen, "step must be positive");
    if (sc->width < 1 || sc->height < 1) return fail(err, errlen, "image size must be positive");
    for (int s = 0; s < sc->n_src; s++) {
        const oracle_source* src = &sc->src[s];
        if (parse_chain(src->chain, src->f_dim, &P->ch[s], err, errlen)) return -1;
        if (oracle_tf_table(src->n_tf, src->tf, P->table[s], err, errlen)) return -1;
    }
    for (int a = 0; a < 3; a++) P->fwd[a] = sc->center[a] - sc->eye[a];
    normalize3(P->fwd);
    cross3(P->fwd, sc->up, P->right);
    normalize3(P->right);
    cross3(P->right, P->fwd, P->upp);
    P->h = sc->orthographic ? 0.5 * sc->ortho_height : tan(0.5 * sc->fovy_deg * ORACLE_PI / 180.0);
    P->aspect = (double)sc->width / (double)sc->height;
    return 0;
}

/* Camera: pixel centres, vertical field of view, row 0 at the top. */
static void pixel_ray(const prepared* P, int i, int j, double o[3], double d[3]) {
    const oracle_scene* sc = P->sc;
    double x = (2.0 * (i + 0.5) / sc->width - 1.0) * P->h * P->aspect;
    double y = (1.0 - 2.0 * (j + 0.5) / sc->height) * P->h;
    if (sc->orthographic) {
        for (int a = 0; a < 3; a++) {
            o[a] = sc->eye[a] + x * P->right[a] + y * P->upp[a];
            d[a] = P->fwd[a];
        }
    } else {
        for (int a = 0; a < 3; a++) {
            o[a] = sc->eye[a];
            d[a] = P->fwd[a] + x * P->right[a] + y * P->upp[a];
        }
        normalize3(d);
    }
}

/* Slab test against the local box [0,N]^3: the interval of t with o + t d inside. */
static int box_interval(const prepared* P, const double o[3], const double d[3], double* t0, double* t1) {
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; a++) {
        double n = (double)P->sc->dims[a];
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > n) return 0;
            continue;
        }
        double ta = (0.0 - o[a]) / d[a];
        double tb = (n - o[a]) / d[a];
        double tn = ta < tb ? ta : tb;
        double tf = ta < tb ? tb : ta;
        if (tn > lo) lo = tn;
        if (tf < hi) hi = tf;
    }
    if (lo < 0.0) lo = 0.0;
    *t0 = lo;
    *t1 = hi;
    return hi > lo;
}

int oracle_ray(const oracle_scene* sc, int i, int j, double o[3], double d[3], double* t0, double* t1) {
    static prepared P;  /* test helper; not re-entrant */
    char err[128];
    oracle_scene tmp = *sc;
    tmp.n_src = 0;
    if (prepare(&tmp, &P, err, sizeof err)) return -1;
    pixel_ray(&P, i, j, o, d);
    return box_interval(&P, o, d, t0, t1);
}

static int clamp_int(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* The chain output of source s at integer cell (x, y, z). */
static double source_value(const prepared* P, int s, int x, int y, int z) {
    const oracle_source* src = &P->sc->src[s];
    const int q[3] = {x, y, z};
    for (int a = 0; a < 3; a++)
        if (q[a] < -src->guard || q[a] > P->sc->dims[a] - 1 + src->guard) {
            /* cannot happen for positions inside the box; never read undeclared memory */
            fprintf(stderr, "oracle: source %d read at index %d on axis %d, outside its guard\n", s, q[a], a);
            abort();
        }
    double v[4];
    for (int c = 0; c < src->f_dim; c++) v[c] = read_component(src, c, x, y, z);
    return apply_chain(&P->ch[s], v, NULL);
}

/* The (interpolated) chain output of source s at position p. */
static double source_at(const prepared* P, int s, const double p[3], const int* cell) {
    const oracle_scene* sc = P->sc;
    const oracle_source* src = &sc->src[s];
    if (sc->interpolation == 0) {
        int q[3];
        for (int a = 0; a < 3; a++)
            q[a] = cell ? cell[a] : clamp_int((int)floor(p[a]), 0, sc->dims[a] - 1);
        return source_value(P, s, q[0], q[1], q[2]);
    }
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; a++) {
        double u = p[a] - 0.5;
        double fl = floor(u);
        i0[a] = (int)fl;
        f[a] = u - fl;
    }
    double x = 0.0;
    for (int corner = 0; corner < 8; corner++) {
        int q[3];
        double w = 1.0;
        for (int a = 0; a < 3; a++) {
            int bit = (corner >> a) & 1;
            q[a] = i0[a] + bit;
            if (src->guard < 1) q[a] = clamp_int(q[a], 0, sc->dims[a] - 1);
            w *= bit ? f[a] : 1.0 - f[a];
        }
        x += w * source_value(P, s, q[0], q[1], q[2]);
    }
    return x;
}

/* One scan point at position p: combined premultiplied colour E and opacity S.
 * cell, when not NULL, overrides the nearest cell (for the flip allowance). */
static void scan_point(const prepared* P, const double p[3], const int* cell, double E[3], double* S) {
    const oracle_scene* sc = P->sc;
    double sumS = 0.0, sumE[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < sc->n_src; s++) {
        const oracle_source* src = &sc->src[s];
        if (!src->enabled) continue;                  /* never read */
        double x = source_at(P, s, p, cell);
        double rgba[4];
        classify(P->table[s], x, rgba);
        double wa = src->weight * rgba[3];
        sumS += wa;
        for (int c = 0; c < 3; c++) sumE[c] += wa * rgba[c];
    }
    if (sumS > 1.0) {
        for (int c = 0; c < 3; c++) sumE[c] /= sumS;
        sumS = 1.0;
    }
    for (int c = 0; c < 3; c++) E[c] = sumE[c];
    *S = sumS;
}

static double max_abs_diff(const double a[3], double as, const double b[3], double bs) {
    double m = 0.0;
    for (int c = 0; c < 3; c++) {
        double v = fabs(a[c] - b[c]);
        if (v > m) m = v;
    }
    return m + fabs(as - bs);
}

/* Is the nearest-cell choice on some axis within delta of an interior cell boundary?
 * Fills alt[] with the other candidate cell per flagged axis; returns the flag mask. */
static int nearest_flags(const prepared* P, const double p[3], int cell[3], int alt[3]) {
    int mask = 0;
    for (int a = 0; a < 3; a++) {
        int n = P->sc->dims[a];
        cell[a] = clamp_int((int)floor(p[a]), 0, n - 1);
        double r = floor(p[a] + 0.5);
        if (r >= 1.0 && r <= (double)(n - 1) && fabs(p[a] - r) < P->sc->delta) {
            mask |= 1 << a;
            alt[a] = (cell[a] == (int)r) ? (int)r - 1 : (int)r;
        }
    }
    return mask;
}

/* The scan point grid: t_k = t0 + (k + 1/2) step. */
static double scan_param(const oracle_scene* sc, double t0, int64_t k) {
    return t0 + ((double)k + 0.5) * sc->step;
}

/* Clipping: keep p iff n.p + d >= 0 for every plane; *near_plane is set when
 * p lies within delta of some plane. */
static int clip_keep(const oracle_scene* sc, const double p[3], int* near_plane) {
    int keep = 1;
    *near_plane = 0;
    for (int c = 0; c < sc->n_clip; c++) {
        const double* pl = sc->clip + 4 * c;
        double s = pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2] + pl[3];
        double nn = sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        if (s < 0.0) keep = 0;
        if (fabs(s) < sc->delta * nn) *near_plane = 1;
    }
    return keep;
}

static void render_pixel(const prepared* P, int i, int j, oracle_pixel* px) {
    const oracle_scene* sc = P->sc;
    memset(px, 0, sizeof(*px));
    double o[3], d[3], t0, t1;
    pixel_ray(P, i, j, o, d);
    if (!box_interval(P, o, d, &t0, &t1)) return;
    double C[3] = {0.0, 0.0, 0.0}, A = 0.0;
    double allowance = 0.0;
    int flags = 0, kinds = 0;
    const double delta = sc->delta;
    for (int64_t k = 0;; k++) {
        double t = scan_param(sc, t0, k);
        int inside = t < t1;
        if (!inside && !(t - t1 < delta)) break;
        double p[3];
        for (int a = 0; a < 3; a++) p[a] = o[a] + t * d[a];
        int near_plane;
        int keep = clip_keep(sc, p, &near_plane) && inside;
        int near_exit = (t1 - t < delta) && (t - t1 < delta);
        int kind = (near_plane ? ORACLE_FLAG_CLIP : 0) | (near_exit ? ORACLE_FLAG_EXIT : 0);
        double T = 1.0 - A;                          /* transmittance before this point */
        if (!keep) {
            if (kind) {                              /* the other side might keep it */
                double E[3], S;
                scan_point(P, p, NULL, E, &S);
                allowance += T * max_abs_diff(E, S, (double[3]){0, 0, 0}, 0.0);
                flags++;
                kinds |= kind;
                px->count_slack++;
            }
            if (!inside) break;
            continue;
        }
        double E[3], S;
        scan_point(P, p, NULL, E, &S);
        if (kind) {                                  /* the other side might drop it */
            allowance += T * max_abs_diff(E, S, (double[3]){0, 0, 0}, 0.0);
            flags++;
            kinds |= kind;
            px->count_slack++;
        }
        if (sc->interpolation == 0) {
            int cell[3], alt[3], mask = nearest_flags(P, p, cell, alt);
            if (mask) {
                double worst = 0.0;
                for (int sub = 1; sub < 8; sub++) {
                    if ((sub & mask) != sub) continue;
                    int q[3];
                    for (int a = 0; a < 3; a++) q[a] = (sub >> a & 1) ? alt[a] : cell[a];
                    double E2[3], S2;
                    scan_point(P, p, q, E2, &S2);
                    double dv = max_abs_diff(E, S, E2, S2);
                    if (dv > worst) worst = dv;
                }
                allowance += T * worst;
                flags++;
                kinds |= ORACLE_FLAG_NEAREST;
            }
        }
        /* classical front-to-back compositing */
        for (int c = 0; c < 3; c++) C[c] = C[c] + (1.0 - A) * E[c];
        A = A + (1.0 - A) * S;
        px->samples++;
        if (A >= sc->ert_threshold) {
            if (A - sc->ert_threshold < sc->ert_margin) {  /* the other side might go on */
                allowance += 1.0 - A;
                flags++;
                kinds |= ORACLE_FLAG_ERT;
            }
            break;
        }
        if (sc->ert_threshold - A < sc->ert_margin) {      /* the other side might stop here */
            allowance += 1.0 - A;
            flags++;
            kinds |= ORACLE_FLAG_ERT;
        }
    }
    for (int c = 0; c < 3; c++) px->rgba[c] = C[c];
    px->rgba[3] = A;
    px->allowance = allowance;
    px->flags = flags;
    px->kinds = kinds;
}

/* ------------------------------------------------------------------ */
/* iso-surface rendering (a listed feature, Sec. 3; no algorithm given): */
/* the surface is the first place along the ray where a source's        */
/* interpolated chain output crosses its iso value between two          */
/* consecutive kept scan points; the crossing is placed by linear        */
/* interpolation, the normal is the central-difference gradient (half a  */
/* voxel), and the opaque pixel is the TF colour at the iso value lit by */
/* a headlight: rgb * (0.3 + 0.7 |n . d|), opacity 1.                    */
/*                                                                       */
/* Decisions within their margins (a kept/dropped scan point near a clip */
/* plane or the box exit, a nearest cell near a boundary, a value near   */
/* the iso value) may go either way in FP32.  The crossing, and with it  */
/* the whole pixel, can move only when the other outcome                 */
/*   - puts some source's value on the other side of its iso value      */
/*     (an iso-margin value; a nearest cell whose alternative lies on    */
/*     the other side; a dropped scan point whose kept value differs in  */
/*     side from a kept neighbour), or                                   */
/*   - changes one of the two scan points the crossing is placed between, */
/*     or a cell the gradient reads;                                     */
/* such a pixel is unconstrained (allowance 2, any sample count).  Other */
/* flagged decisions only move the count by one (a kept scan point that  */
/* might be dropped, or the reverse, away from the crossing).            */
/* ------------------------------------------------------------------ */
#define ISO_FREE_COUNT (1 << 30)

/* side of each surfaced source's value: bit s set when x[s] >= iso */
static unsigned iso_sides(const prepared* P, const double* x) {
    unsigned m = 0;
    for (int s = 0; s < P->sc->n_src; s++) {
        const oracle_source* src = &P->sc->src[s];
        if (!src->enabled || isnan(src->iso)) continue;
        if (x[s] >= src->iso) m |= 1u << s;
    }
    return m;
}

static void iso_values(const prepared* P, const double p[3], const int* cell, double* x) {
    for (int s = 0; s < P->sc->n_src; s++) {
        const oracle_source* src = &P->sc->src[s];
        x[s] = 0.0;
        if (!src->enabled || isnan(src->iso)) continue;
        x[s] = source_at(P, s, p, cell);
    }
}

/* How far source s's value at p can move in FP32 evaluation: the position
 * may be off by up to delta voxels per axis (the value then moves by at most
 * the larger change over +-delta along each axis, summed over the axes; the
 * interpolant is multilinear per cell), and the arithmetic by a small
 * relative amount (iso_margin relative to the value's magnitude). */
static double iso_value_margin(const prepared* P, int s, const double p[3], double x) {
    double m = 0.0;
    for (int a = 0; a < 3; a++) {
        double q[3] = {p[0], p[1], p[2]};
        q[a] = p[a] + P->sc->delta;
        double up = fabs(source_at(P, s, q, NULL) - x);
        q[a] = p[a] - P->sc->delta;
        double dn = fabs(source_at(P, s, q, NULL) - x);
        m += up > dn ? up : dn;
    }
    return m + P->sc->iso_margin * (1.0 + fabs(x));
}

static void iso_pixel(const prepared* P, int i, int j, oracle_pixel* px) {
    const oracle_scene* sc = P->sc;
    memset(px, 0, sizeof(*px));
    double o[3], d[3], t0, t1;
    pixel_ray(P, i, j, o, d);
    if (!box_interval(P, o, d, &t0, &t1)) return;
    const double delta = sc->delta;
    double prev[MAX_SRC];
    double t_prev = 0.0;
    int have_prev = 0;
    int unconstrained = 0;        /* some flagged decision can move the crossing */
    int prev_flagged = 0;         /* the scan point held in prev[] carries a flagged decision */
    int pending = 0;              /* a flagged dropped point whose kept value's sides are in pending_sides */
    unsigned pending_sides = 0;
    for (int64_t k = 0;; k++) {
        double t = scan_param(sc, t0, k);
        int inside = t < t1;
        if (!inside && !(t - t1 < delta)) break;
        double p[3];
        for (int a = 0; a < 3; a++) p[a] = o[a] + t * d[a];
        int near_plane;
        int keep = clip_keep(sc, p, &near_plane) && inside;
        int near_exit = (t1 - t < delta) && (t - t1 < delta);
        int kind = (near_plane ? ORACLE_FLAG_CLIP : 0) | (near_exit ? ORACLE_FLAG_EXIT : 0);
        if (!keep) {
            if (kind) {
                /* kept on the other side: it joins the chain of kept points around it */
                double xa[MAX_SRC];
                iso_values(P, p, NULL, xa);
                unsigned alt = iso_sides(P, xa);
                if (have_prev && alt != iso_sides(P, prev)) unconstrained = 1;
                pending = 1;
                pending_sides = alt;
                px->flags++;
                px->kinds |= kind;
                px->count_slack++;
            } else {
                pending = 0;
            }
            have_prev = 0;
            prev_flagged = 0;
            if (!inside) break;
            continue;
        }
        int flagged_here = 0;
        if (kind) {                                   /* the other side might drop it */
            px->flags++;
            px->kinds |= kind;
            px->count_slack++;
            flagged_here = 1;
        }
        double x[MAX_SRC];
        iso_values(P, p, NULL, x);
        const unsigned sides = iso_sides(P, x);
        if (sc->interpolation == 0) {
            int cell[3], alt[3], mask = nearest_flags(P, p, cell, alt);
            if (mask) {
                px->flags++;
                px->kinds |= ORACLE_FLAG_NEAREST;
                flagged_here = 1;
                for (int sub = 1; sub < 8; sub++) {
                    if ((sub & mask) != sub) continue;
                    int q[3];
                    for (int a = 0; a < 3; a++) q[a] = (sub >> a & 1) ? alt[a] : cell[a];
                    double xa[MAX_SRC];
                    iso_values(P, p, q, xa);
                    if (iso_sides(P, xa) != sides) unconstrained = 1;
                }
            }
        }
        for (int s = 0; s < sc->n_src; s++) {
            const oracle_source* src = &sc->src[s];
            if (!src->enabled || isnan(src->iso)) continue;
            if (fabs(x[s] - src->iso) < iso_value_margin(P, s, p, x[s])) {
                px->kinds |= ORACLE_FLAG_ISO;
                px->flags++;
                unconstrained = 1;
            }
        }
        if (pending && sides != pending_sides) unconstrained = 1;
        pending = 0;
        px->samples++;
        int hit = -1;
        double f = 0.0;
        for (int s = 0; s < sc->n_src; s++) {
            const oracle_source* src = &sc->src[s];
            if (!src->enabled || isnan(src->iso)) continue;
            if (hit < 0 && have_prev && ((prev[s] >= src->iso) != (x[s] >= src->iso))) {
                hit = s;
                f = (src->iso - prev[s]) / (x[s] - prev[s]);
            }
        }
        if (hit >= 0) {
            /* a flagged decision at either end of the crossing moves it */
            if (flagged_here || prev_flagged) unconstrained = 1;
            const oracle_source* src = &sc->src[hit];
            double ts = t_prev + f * (t - t_prev), q[3], g[3];
            for (int a = 0; a < 3; a++) q[a] = o[a] + ts * d[a];
            for (int a = 0; a < 3; a++) {
                double qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
                qp[a] += 0.5;
                qm[a] -= 0.5;
                if (sc->interpolation == 0) {
                    int c1[3], a1[3], c2[3], a2[3];
                    if (nearest_flags(P, qp, c1, a1) || nearest_flags(P, qm, c2, a2)) {
                        px->flags++;
                        px->kinds |= ORACLE_FLAG_NEAREST;
                        unconstrained = 1;
                    }
                }
                g[a] = source_at(P, hit, qp, NULL) - source_at(P, hit, qm, NULL);
            }
            double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            double cosine = gl > 0.0 ? fabs(g[0] * d[0] + g[1] * d[1] + g[2] * d[2]) / gl : 1.0;
            double rgba[4];
            classify(P->table[hit], src->iso, rgba);
            double light = 0.3 + 0.7 * cosine;
            for (int c = 0; c < 3; c++) px->rgba[c] = rgba[c] * light;
            px->rgba[3] = 1.0;
            break;
        }
        for (int s = 0; s < sc->n_src; s++) prev[s] = x[s];
        t_prev = t;
        have_prev = 1;
        prev_flagged = flagged_here;
    }
    if (unconstrained) {
        px->allowance = 2.0;
        px->count_slack = ISO_FREE_COUNT;
    }
}

static int check_scene(const oracle_scene* sc, char* err, int errlen) {
    for (int s = 0; s < sc->n_src; s++) {
        const oracle_source* src = &sc->src[s];
        if (!src->enabled) continue;
        if (src->f_dim < 1 || src->f_dim > 4) return fail(err, errlen, "source %d: f_dim outside 1..4", s);
        if (src->dtype < 0 || src->dtype > 2) return fail(err, errlen, "source %d: bad dtype", s);
        for (int c = 0; c < src->f_dim; c++)
            if (!src->comp[c]) return fail(err, errlen, "source %d: null component pointer", s);
    }
    return 0;
}

int oracle_render_range(const oracle_scene* sc, int64_t first, int64_t count, oracle_pixel* out,
                        char* err, int errlen) {
    prepared* P = (prepared*)malloc(sizeof(prepared));
    if (!P) return fail(err, errlen, "out of memory");
    if (check_scene(sc, err, errlen) || prepare(sc, P, err, errlen)) {
        free(P);
        return -1;
    }
    int64_t total = (int64_t)sc->width * sc->height;
    for (int64_t q = 0; q < count; q++) {
        int64_t idx = first + q;
        if (idx < 0 || idx >= total) {
            free(P);
            return fail(err, errlen, "pixel index out of range");
        }
        if (sc->mode == 1) iso_pixel(P, (int)(idx % sc->width), (int)(idx / sc->width), &out[q]);
        else render_pixel(P, (int)(idx % sc->width), (int)(idx / sc->width), &out[q]);
    }
    free(P);
    return 0;
}

int oracle_render_list(const oracle_scene* sc, const int32_t* px, int64_t n, oracle_pixel* out,
                       char* err, int errlen) {
    prepared* P = (prepared*)malloc(sizeof(prepared));
    if (!P) return fail(err, errlen, "out of memory");
    if (check_scene(sc, err, errlen) || prepare(sc, P, err, errlen)) {
        free(P);
        return -1;
    }
    for (int64_t q = 0; q < n; q++) {
        int i = px[2 * q], j = px[2 * q + 1];
        if (i < 0 || i >= sc->width || j < 0 || j >= sc->height) {
            free(P);
            return fail(err, errlen, "pixel (%d,%d) outside the image", i, j);
        }
        if (sc->mode == 1) iso_pixel(P, i, j, &out[q]);
        else render_pixel(P, i, j, &out[q]);
    }
    free(P);
    return 0;
}

/* ------------------------------------------------------------------ */
/* frame encode: FP32, one rounding per operation (no contraction)      */
/* ------------------------------------------------------------------ */
static unsigned char quantize_channel(float v) {
    float c;
    if (isnan(v) || v <= 0.0f) c = 0.0f;
    else if (v >= 1.0f) c = 1.0f;
    else c = v;
    float scaled = c * 255.0f;
    float shifted = scaled + 0.5f;
    return (unsigned char)floorf(shifted);
}

void oracle_encode_rgba8(const float* rgba, int64_t n_pixels, const float* background, unsigned char* out) {
    for (int64_t i = 0; i < n_pixels; i++) {
        const float* px = rgba + 4 * i;
        unsigned char* q = out + 4 * i;
        if (background) {
            float transmit = 1.0f - px[3];
            for (int c = 0; c < 3; c++) {
                float behind = transmit * background[c];
                q[c] = quantize_channel(px[c] + behind);
            }
            q[3] = 255;
        } else {
            for (int c = 0; c < 4; c++) q[c] = quantize_channel(px[c]);
        }
    }
}
