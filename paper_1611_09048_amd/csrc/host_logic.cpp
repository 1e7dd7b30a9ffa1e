// Host-only logic of the library (no HIP calls); see host_logic.h.
#include "host_logic.h"

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <vector>

namespace isaac {
namespace host {

namespace {
constexpr double kPi = 3.14159265358979323846;
}

// ---------------------------------------------------------------------------
// functor chains: "name(args) | name | ..." (Sec. 3.3, Tab. "functors")
// ---------------------------------------------------------------------------
bool compile_chain(const char* text, int f_dim, CompiledChain& out, std::string& err) {
    out = CompiledChain();
    if (f_dim < 1 || f_dim > 4) {
        err = "f_dim must be 1..4";
        return false;
    }
    int dim = f_dim;
    std::vector<DevOp> ops;
    const char* s = text ? text : "";
    auto ws = [&]() { while (*s == ' ' || *s == '\t' || *s == '\n' || *s == '\r') ++s; };
    ws();
    int parsed = 0;
    while (*s) {
        if (parsed > 0) {
            if (*s != '|') {
                err = std::string("expected '|' before: ") + s;
                return false;
            }
            ++s;
            ws();
        }
        std::string name;
        while (*s && std::isalpha((unsigned char)*s)) name.push_back(*s++);
        ws();
        std::vector<double> args;
        bool parens = false;
        if (*s == '(') {
            parens = true;
            ++s;
            ws();
            while (*s != ')') {
                char* end = nullptr;
                double v = std::strtod(s, &end);
                if (end == s) {
                    err = "expected a number in the arguments of '" + name + "'";
                    return false;
                }
                args.push_back(v);
                s = end;
                ws();
                if (*s == ',') {
                    ++s;
                    ws();
                    if (*s == ')') {
                        err = "dangling ',' in '" + name + "'";
                        return false;
                    }
                } else if (*s != ')') {
                    err = "expected ',' or ')' in '" + name + "'";
                    return false;
                }
            }
            ++s;
            ws();
        }
        (void)parens;
        DevOp op{};
        op.dim = dim;
        if (name == "add" || name == "mul" || name == "pow") {
            if (args.size() != 1 && (int)args.size() != dim) {
                err = "'" + name + "' takes 1 or " + std::to_string(dim) + " arguments, got " +
                      std::to_string(args.size());
                return false;
            }
            op.kind = name == "add" ? OP_ADD : name == "mul" ? OP_MUL : OP_POW;
            for (int c = 0; c < 4; ++c) op.arg[c] = (float)(args.size() == 1 ? args[0] : (c < dim ? args[c] : 0.0));
        } else if (name == "length" || name == "sum") {
            if (!args.empty()) {
                err = "'" + name + "' takes no arguments";
                return false;
            }
            op.kind = name == "length" ? OP_LENGTH : OP_SUM;
            dim = 1;
        } else {
            err = name.empty() ? std::string("expected a functor name before: ") + s
                               : "unknown functor '" + name + "'";
            return false;
        }
        ops.push_back(op);
        ++parsed;
        if (parsed > kMaxOps) {
            err = "more than " + std::to_string(kMaxOps) + " functors";
            return false;
        }
    }
    // host-side simplification; every rewrite is exact in IEEE arithmetic
    // except pow(x, 0.5) -> sqrt(x), which differs only for -0 and -inf
    std::vector<DevOp> simp;
    for (const DevOp& op : ops) {
        bool all_eq = true;
        for (int c = 1; c < op.dim; ++c) all_eq = all_eq && op.arg[c] == op.arg[0];
        if ((op.kind == OP_MUL || op.kind == OP_POW) && all_eq && op.arg[0] == 1.0f) continue;
        if (op.kind == OP_ADD && all_eq && op.arg[0] == 0.0f) continue;
        DevOp o = op;
        if (op.kind == OP_POW && all_eq && op.arg[0] == 0.5f) o.kind = OP_SQRT;
        if (op.kind == OP_POW && all_eq && op.arg[0] == 2.0f) o.kind = OP_SQUARE;
        simp.push_back(o);
    }
    out.n_ops = (int)simp.size();
    for (int i = 0; i < out.n_ops; ++i) out.ops[i] = simp[i];
    out.out_dim = dim;
    return true;
}

// ---------------------------------------------------------------------------
// transfer tables: T[j] = PL(j / 255), j = 0..255
// ---------------------------------------------------------------------------
bool bake_tf(const isaac_tf_point* pts, int n, float* table, std::string& err) {
    if (!pts || n < 2) {
        err = "a transfer function needs at least 2 points";
        return false;
    }
    if (pts[0].x != 0.0 || pts[n - 1].x != 1.0) {
        err = "transfer function points must start at x=0 and end at x=1";
        return false;
    }
    for (int i = 0; i < n; ++i) {
        if (i > 0 && !(pts[i].x > pts[i - 1].x)) {
            err = "transfer function x must increase strictly";
            return false;
        }
        for (int c = 0; c < 4; ++c)
            if (!(pts[i].rgba[c] >= 0.0 && pts[i].rgba[c] <= 1.0)) {
                err = "transfer function values must lie in [0,1]";
                return false;
            }
    }
    int seg = 0;
    for (int j = 0; j < kTfEntries; ++j) {
        const double x = (double)j / 255.0;
        while (seg < n - 2 && x > pts[seg + 1].x) ++seg;
        const isaac_tf_point& a = pts[seg];
        const isaac_tf_point& b = pts[seg + 1];
        const double w = (x - a.x) / (b.x - a.x);
        for (int c = 0; c < 4; ++c) table[4 * j + c] = (float)(a.rgba[c] + w * (b.rgba[c] - a.rgba[c]));
    }
    return true;
}

bool camera_basis(const isaac_render_desc& j, CameraBasis& cb, std::string& err) {
    double f[3] = {j.center[0] - j.eye[0], j.center[1] - j.eye[1], j.center[2] - j.eye[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0) || !std::isfinite(fl)) {
        err = "eye and center must differ";
        return false;
    }
    for (int a = 0; a < 3; ++a) cb.fwd[a] = f[a] / fl;
    const double* u = j.up;
    double r[3] = {cb.fwd[1] * u[2] - cb.fwd[2] * u[1], cb.fwd[2] * u[0] - cb.fwd[0] * u[2],
                   cb.fwd[0] * u[1] - cb.fwd[1] * u[0]};
    // |fwd x up| = |up| sin(angle): an up within 1e-6 rad of the view direction
    // leaves only rounding noise in the cross product (no usable right vector)
    const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!std::isfinite(rl) || !std::isfinite(ul) || !(rl > 1e-6 * ul)) {
        err = "up must be finite and not parallel to the view direction";
        return false;
    }
    for (int a = 0; a < 3; ++a) cb.right[a] = r[a] / rl;
    cb.upp[0] = cb.right[1] * cb.fwd[2] - cb.right[2] * cb.fwd[1];
    cb.upp[1] = cb.right[2] * cb.fwd[0] - cb.right[0] * cb.fwd[2];
    cb.upp[2] = cb.right[0] * cb.fwd[1] - cb.right[1] * cb.fwd[0];
    if (j.projection == ISAAC_ORTHOGRAPHIC) {
        cb.h = 0.5 * j.ortho_height;
    } else {
        cb.h = std::tan(0.5 * j.fovy_deg * kPi / 180.0);
    }
    cb.aspect = (double)j.width / (double)j.height;
    return true;
}

// A pixel rectangle containing every pixel whose ray can meet the box (the
// local box, or the brick's box in the global index space): the projections
// of the 8 box corners bound the projection of the convex box, widened by one
// pixel.  A corner at or behind the eye plane disables the test.
void set_cull_rect(DevJob& dj) {
    dj.cull[0] = 0;
    dj.cull[1] = 0;
    dj.cull[2] = dj.width - 1;
    dj.cull[3] = dj.height - 1;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = dj.org[a];
        hi[a] = (double)dj.org[a] + dj.dims[a];
    }
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int c = 0; c < 8; ++c) {
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = ((c >> a) & 1 ? hi[a] : lo[a]) - dj.eye[a];
        const double vr = v[0] * dj.right[0] + v[1] * dj.right[1] + v[2] * dj.right[2];
        const double vu = v[0] * dj.upp[0] + v[1] * dj.upp[1] + v[2] * dj.upp[2];
        double x, y;
        if (dj.ortho) {
            x = vr / (dj.h * dj.aspect);
            y = vu / dj.h;
        } else {
            const double z = v[0] * dj.fwd[0] + v[1] * dj.fwd[1] + v[2] * dj.fwd[2];
            const double vl = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(z > 1e-6 * (vl + 1.0))) return;
            x = vr / (z * dj.h * dj.aspect);
            y = vu / (z * dj.h);
        }
        const double pi = (x + 1.0) * 0.5 * dj.width - 0.5;
        const double pj = (1.0 - y) * 0.5 * dj.height - 0.5;
        xmin = std::min(xmin, pi);
        xmax = std::max(xmax, pi);
        ymin = std::min(ymin, pj);
        ymax = std::max(ymax, pj);
    }
    auto clampd = [](double v, double a, double b) { return std::min(std::max(v, a), b); };
    dj.cull[0] = (int)clampd(std::floor(xmin) - 1.0, 0.0, (double)dj.width);
    dj.cull[1] = (int)clampd(std::floor(ymin) - 1.0, 0.0, (double)dj.height);
    dj.cull[2] = (int)clampd(std::ceil(xmax) + 1.0, -1.0, (double)dj.width - 1);
    dj.cull[3] = (int)clampd(std::ceil(ymax) + 1.0, -1.0, (double)dj.height - 1);
}

}  // namespace host
}  // namespace isaac
