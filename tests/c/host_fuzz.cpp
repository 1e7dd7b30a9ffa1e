// Sanitizer harness for the library's host-only logic (chain compiler,
// transfer-table bake, camera basis, screen rectangle): seeded random and
// hostile inputs, with the invariants each function promises checked on every
// accepted input.  Built with -fsanitize=address,undefined by
// tests/test_host_sanitizers.py and run on the CPU; exit 0 when every check
// holds and the sanitizers report nothing.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "host_logic.h"

using namespace isaac;
using namespace isaac::host;

static int failures = 0;
#define CHECK(cond, ...)                             \
    do {                                             \
        if (!(cond)) {                               \
            std::fprintf(stderr, "FAIL %s: ", #cond); \
            std::fprintf(stderr, __VA_ARGS__);       \
            std::fprintf(stderr, "\n");              \
            ++failures;                              \
        }                                            \
    } while (0)

static std::mt19937_64 rng(20161128);
static double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }
static int pick(int n) { return (int)(rng() % (uint64_t)n); }

static std::string random_chain() {
    static const char* toks[] = {"add", "mul", "pow", "length", "sum", "sqrt", "", "x", "(", ")", ",", "|", " ",
                                 "\t", "1", "-2.5", "0", "0.5", "2", "1e400", "nan", "inf", "-inf", "1e-300",
                                 "3,4", "(1)", "(1,2,3)", "(1,2,3,4,5)", "||", "length(1)", "\xff", "\x01", "mul(",
                                 "add(1,", ")("};
    std::string s;
    const int n = pick(24);
    for (int i = 0; i < n; ++i) s += toks[pick((int)(sizeof toks / sizeof *toks))];
    return s;
}

static void fuzz_chains() {
    // the paper's worked chains parse with the documented dimensions
    CompiledChain c;
    std::string err;
    CHECK(compile_chain("mul(2,3,4) | add(1) | length", 3, c, err) && c.out_dim == 1 && c.n_ops == 3, "%s", err.c_str());
    CHECK(compile_chain("mul(0,1,0) | sum", 3, c, err) && c.out_dim == 1, "%s", err.c_str());
    CHECK(compile_chain("", 4, c, err) && c.out_dim == 4 && c.n_ops == 0, "identity");
    CHECK(compile_chain(nullptr, 2, c, err) && c.n_ops == 0, "null chain");
    CHECK(!compile_chain("length", 0, c, err) && !compile_chain("length", 5, c, err), "f_dim range");
    CHECK(!compile_chain("add(1)|add(1)|add(1)|add(1)|add(1)|add(1)|add(1)|add(1)|add(1)", 1, c, err), "> 8 ops");
    // a very long chain and a long run of one character
    std::string longc;
    for (int i = 0; i < 5000; ++i) longc += "mul(1.5)|";
    CHECK(!compile_chain(longc.c_str(), 1, c, err), "long chain");
    std::string parens(100000, '(');
    CHECK(!compile_chain(parens.c_str(), 1, c, err), "parens");
    for (int it = 0; it < 200000; ++it) {
        const std::string s = random_chain();
        const int f = pick(6);
        CompiledChain out;
        std::string e;
        const bool ok = compile_chain(s.c_str(), f, out, e);
        if (ok) {
            CHECK(f >= 1 && f <= 4, "accepted f_dim %d", f);
            CHECK(out.n_ops >= 0 && out.n_ops <= kMaxOps, "n_ops %d for '%s'", out.n_ops, s.c_str());
            CHECK(out.out_dim >= 1 && out.out_dim <= f, "out_dim %d for '%s'", out.out_dim, s.c_str());
            for (int i = 0; i < out.n_ops; ++i) {
                CHECK(out.ops[i].kind >= OP_ADD && out.ops[i].kind <= OP_SQUARE, "kind");
                CHECK(out.ops[i].dim >= 1 && out.ops[i].dim <= 4, "dim");
            }
        } else {
            CHECK(!e.empty(), "rejected without a message: '%s'", s.c_str());
        }
    }
}

static void fuzz_tables() {
    const double special[] = {0.0, 1.0, 0.5, -0.0, -1e-300, 1.0 + 1e-15, std::numeric_limits<double>::quiet_NaN(),
                              std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity(),
                              1e300, 0.25, 0.75};
    float table[256 * 4];
    std::string err;
    CHECK(!bake_tf(nullptr, 4, table, err), "null points");
    for (int it = 0; it < 50000; ++it) {
        const int n = pick(12) == 0 ? pick(400) : pick(10);
        std::vector<isaac_tf_point> p((size_t)std::max(n, 1));
        double x = 0.0;
        for (int i = 0; i < n; ++i) {
            const int mode = pick(10);
            if (mode == 0) p[i].x = special[pick(12)];
            else if (mode == 1) p[i].x = x;                             // repeated x
            else p[i].x = x = (i == 0 ? 0.0 : std::min(1.0, x + unif(0.0, 0.4)));
            if (i == n - 1 && pick(3)) p[i].x = 1.0;
            for (int c = 0; c < 4; ++c) p[i].rgba[c] = pick(15) == 0 ? special[pick(12)] : unif(0.0, 1.0);
        }
        std::string e;
        if (bake_tf(n > 0 ? p.data() : nullptr, n, table, e)) {
            CHECK(n >= 2 && p[0].x == 0.0 && p[n - 1].x == 1.0, "accepted bad span");
            for (int i = 1; i < n; ++i) CHECK(p[i].x > p[i - 1].x, "accepted unsorted");
            for (int k = 0; k < 256 * 4; ++k) CHECK(table[k] >= 0.0f && table[k] <= 1.0f, "table value %g", table[k]);
            // the table interpolates the points it passes through
            for (int i = 0; i < n; ++i) {
                const double u = p[i].x * 255.0;
                if (u == std::floor(u))
                    for (int c = 0; c < 4; ++c)
                        CHECK(std::fabs(table[4 * (int)u + c] - p[i].rgba[c]) < 1e-6, "control point %d", i);
            }
        } else {
            CHECK(!e.empty(), "rejected without a message");
        }
    }
}

static isaac_render_desc random_job() {
    isaac_render_desc j;
    std::memset(&j, 0, sizeof j);
    const double big = pick(20) == 0 ? 1e300 : 200.0;
    for (int a = 0; a < 3; ++a) {
        j.eye[a] = unif(-big, big);
        j.center[a] = pick(10) == 0 ? j.eye[a] : unif(-big, big);
        j.up[a] = pick(8) == 0 ? 0.0 : unif(-1.0, 1.0);
    }
    if (pick(10) == 0)
        for (int a = 0; a < 3; ++a) j.up[a] = j.center[a] - j.eye[a];   // parallel to the view
    if (pick(30) == 0) j.eye[pick(3)] = std::numeric_limits<double>::quiet_NaN();
    j.projection = pick(4) == 0 ? ISAAC_ORTHOGRAPHIC : ISAAC_PERSPECTIVE;
    j.fovy_deg = unif(1.0, 170.0);
    j.ortho_height = unif(1.0, 500.0);
    j.width = 1 + pick(4096);
    j.height = 1 + pick(4096);
    return j;
}

static void fuzz_cameras() {
    for (int it = 0; it < 200000; ++it) {
        const isaac_render_desc j = random_job();
        CameraBasis cb;
        std::string e;
        if (!camera_basis(j, cb, e)) {
            CHECK(!e.empty(), "rejected without a message");
            continue;
        }
        const double* v[3] = {cb.fwd, cb.right, cb.upp};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double d = v[a][0] * v[b][0] + v[a][1] * v[b][1] + v[a][2] * v[b][2];
                CHECK(std::isfinite(d) && std::fabs(d - (a == b ? 1.0 : 0.0)) < 1e-9, "basis %d.%d = %g", a, b, d);
            }
        CHECK(std::isfinite(cb.h) && cb.h > 0.0 && cb.aspect > 0.0, "h %g", cb.h);
        // the screen rectangle of a random box stays inside the image
        DevJob dj;
        std::memset(&dj, 0, sizeof dj);
        for (int a = 0; a < 3; ++a) {
            dj.eye[a] = j.eye[a];
            dj.fwd[a] = cb.fwd[a];
            dj.right[a] = cb.right[a];
            dj.upp[a] = cb.upp[a];
            dj.dims[a] = 1 + pick(1024);
            dj.org[a] = (float)(pick(4) == 0 ? pick(512) : 0);
        }
        dj.h = cb.h;
        dj.aspect = cb.aspect;
        dj.ortho = j.projection == ISAAC_ORTHOGRAPHIC;
        dj.width = j.width;
        dj.height = j.height;
        set_cull_rect(dj);
        CHECK(dj.cull[0] >= 0 && dj.cull[1] >= 0 && dj.cull[2] <= dj.width - 1 && dj.cull[3] <= dj.height - 1 &&
                  dj.cull[2] >= -1 && dj.cull[3] >= -1 && dj.cull[0] <= dj.width && dj.cull[1] <= dj.height,
              "cull %d %d %d %d of %dx%d", dj.cull[0], dj.cull[1], dj.cull[2], dj.cull[3], dj.width, dj.height);
    }
}

int main() {
    fuzz_chains();
    fuzz_tables();
    fuzz_cameras();
    std::printf("host fuzz: %d failures\n", failures);
    return failures ? 1 : 0;
}
