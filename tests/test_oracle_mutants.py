"""Plant plausible mistakes in a copy of the oracle and check that a pin catches each.

Every mutant is one textual change to oracle/isaac_oracle.c (a dropped term, a
wrong sign, an off-by-one, a transposed operand ...).  The copy is compiled
to a temporary library and the full pin suite runs against it in a child
process (a mutant may also crash, which counts as caught).  A mutant that
passes every pin means the pins do not constrain that part of the oracle.
"""

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "isaac_oracle.c")

MUTANTS = [
    ("composite_drops_transmittance", "C[c] = C[c] + (1.0 - A) * E[c];", "C[c] = C[c] + E[c];"),
    ("alpha_drops_transmittance", "A = A + (1.0 - A) * S;", "A = A + S;"),
    ("grid_not_half_step", "t0 + ((double)k + 0.5) * sc->step", "t0 + ((double)k) * sc->step"),
    ("trilinear_vertex_centred", "double u = p[a] - 0.5;", "double u = p[a];"),
    ("trilinear_weights_swapped", "w *= bit ? f[a] : 1.0 - f[a];", "w *= bit ? 1.0 - f[a] : f[a];"),
    ("chain_last_component", "    return v[0];\n}", "    return v[dim - 1];\n}"),
    ("add_no_broadcast", "v[k] = v[k] + (f->nargs == 1 ? f->arg[0] : f->arg[k]);", "v[k] = v[k] + f->arg[k];"),
    ("mul_no_broadcast", "v[k] = v[k] * (f->nargs == 1 ? f->arg[0] : f->arg[k]);", "v[k] = v[k] * f->arg[k];"),
    ("pow_operands_swapped", "pow(v[k], f->nargs == 1 ? f->arg[0] : f->arg[k])",
     "pow(f->nargs == 1 ? f->arg[0] : f->arg[k], v[k])"),
    ("length_without_square", "s += v[k] * v[k];", "s += v[k] * v[k] * v[k];"),
    ("sum_of_squares", "for (int k = 0; k < dim; k++) s += v[k];\n", "for (int k = 0; k < dim; k++) s += v[k] * v[k];\n"),
    ("tf_scale_256", "double u = 255.0 * t;", "double u = 256.0 * t;"),
    ("tf_no_lerp", "rgba[c] = table[4 * j + c] + f * (table[4 * (j + 1) + c] - table[4 * j + c]);",
     "rgba[c] = table[4 * j + c];"),
    ("tf_index_cap", "if (j > 254) j = 254;", "if (j > 253) j = 253;"),
    ("nan_not_zero", "double t = isnan(x) ? 0.0 :", "double t = isnan(x) ? 1.0 :"),
    ("pl_wrong_weight", "double w = (x - x0) / (x1 - x0);", "double w = (x - x0) / x1;"),
    ("mix_no_saturation", "if (sumS > 1.0) {", "if (sumS > 2.0) {"),
    ("mix_not_renormalised", "sumE[c] /= sumS;", "sumE[c] /= 1.0;"),
    ("weight_dropped", "double wa = src->weight * rgba[3];", "double wa = rgba[3];"),
    ("clip_side_flipped", "if (s < 0.0) keep = 0;", "if (s > 0.0) keep = 0;"),
    ("eye_inside_not_clamped", "if (lo < 0.0) lo = 0.0;", "if (lo < -1e300) lo = 0.0;"),
    ("camera_left_handed", "cross3(P->fwd, sc->up, P->right);", "cross3(sc->up, P->fwd, P->right);"),
    ("image_upside_down", "double y = (1.0 - 2.0 * (j + 0.5) / sc->height) * P->h;",
     "double y = (2.0 * (j + 0.5) / sc->height - 1.0) * P->h;"),
    ("no_aspect", "* P->h * P->aspect;", "* P->h;"),
    ("fovy_not_halved", "tan(0.5 * sc->fovy_deg * ORACLE_PI / 180.0)", "tan(sc->fovy_deg * ORACLE_PI / 180.0)"),
    ("ortho_origin_fixed", "o[a] = sc->eye[a] + x * P->right[a] + y * P->upp[a];", "o[a] = sc->eye[a];"),
    ("strides_transposed", "(int64_t)x * s->stride[0] + (int64_t)y * s->stride[1]",
     "(int64_t)x * s->stride[1] + (int64_t)y * s->stride[0]"),
    ("guard_ignored", "if (src->guard < 1) q[a] = clamp_int(", "if (src->guard < 2) q[a] = clamp_int("),
    ("disabled_read", "        if (!src->enabled) continue;                  /* never read */\n", ""),
    ("ert_strict", "if (A >= sc->ert_threshold) {", "if (A > sc->ert_threshold + 1e-3) {"),
    ("nearest_rounds", "cell ? cell[a] : clamp_int((int)floor(p[a]), 0, sc->dims[a] - 1);",
     "cell ? cell[a] : clamp_int((int)floor(p[a] + 0.5), 0, sc->dims[a] - 1);"),
    ("half_exponent_bias", "e - 25);", "e - 24);"),
    ("bf16_shift", "(uint32_t)b << 16;", "(uint32_t)b << 15;"),
    ("parallel_slab_open", "if (o[a] < 0.0 || o[a] > n) return 0;", "if (o[a] < 0.0) return 0;"),
    ("exit_inclusive", "const double delta = sc->delta;\n    for (int64_t k = 0;; k++) {\n        double t = scan_param(sc, t0, k);\n        int inside = t < t1;",
     "const double delta = sc->delta;\n    for (int64_t k = 0;; k++) {\n        double t = scan_param(sc, t0, k);\n        int inside = t <= t1 + 0.25;"),
    ("iso_midpoint", "f = (src->iso - prev[s]) / (x[s] - prev[s]);", "f = 0.5;"),
    ("iso_refine_from_far_end", "double ts = t_prev + f * (t - t_prev)", "double ts = t - f * (t - t_prev)"),
    ("iso_light_swapped", "double light = 0.3 + 0.7 * cosine;", "double light = 0.7 + 0.3 * cosine;"),
    ("iso_colour_of_sample", "classify(P->table[hit], src->iso, rgba);", "classify(P->table[hit], x[hit], rgba);"),
    ("iso_rising_only", "((prev[s] >= src->iso) != (x[s] >= src->iso))", "(prev[s] < src->iso && x[s] >= src->iso)"),
    ("iso_gradient_skewed", "qm[a] -= 0.5;", "qm[(a + 1) % 3] -= 0.5;"),
    ("encode_truncates", "float shifted = scaled + 0.5f;", "float shifted = scaled;"),
    ("encode_scale_256", "float scaled = c * 255.0f;", "float scaled = c * 256.0f;"),
    ("encode_alpha_as_transmittance", "float transmit = 1.0f - px[3];", "float transmit = px[3];"),
    ("encode_alpha_kept_over_bg", "q[3] = 255;", "q[3] = quantize_channel(px[3]);"),
    ("iso_translucent", "px->rgba[3] = 1.0;\n            break;", "px->rgba[3] = 0.5;\n            break;"),
    # the several-correct-results bookkeeping (decisions within their margins)
    ("nearest_margin_x100", "fabs(p[a] - r) < P->sc->delta", "fabs(p[a] - r) < 100.0 * P->sc->delta"),
    ("nearest_alternative_same_cell", "alt[a] = (cell[a] == (int)r) ? (int)r - 1 : (int)r;", "alt[a] = cell[a];"),
    ("nearest_allowance_without_T", "allowance += T * worst;", "allowance += worst;"),
    ("every_point_flagged_clip",
     "int kind = (near_plane ? ORACLE_FLAG_CLIP : 0) | (near_exit ? ORACLE_FLAG_EXIT : 0);\n        double T",
     "int kind = ORACLE_FLAG_CLIP | (near_exit ? ORACLE_FLAG_EXIT : 0);\n        double T"),
    ("clip_margin_unnormalised", "if (fabs(s) < sc->delta * nn) *near_plane = 1;",
     "if (fabs(s) < sc->delta) *near_plane = 1;"),
    ("exit_never_flagged",
     "int near_exit = (t1 - t < delta) && (t - t1 < delta);\n"
     "        int kind = (near_plane ? ORACLE_FLAG_CLIP : 0) | (near_exit ? ORACLE_FLAG_EXIT : 0);\n        double T",
     "int near_exit = 0;\n"
     "        int kind = (near_plane ? ORACLE_FLAG_CLIP : 0) | (near_exit ? ORACLE_FLAG_EXIT : 0);\n        double T"),
    ("kept_flag_without_T",
     "/* the other side might drop it */\n            allowance += T * max_abs_diff",
     "/* the other side might drop it */\n            allowance += max_abs_diff"),
    ("count_slack_inflated",
     "/* the other side might drop it */\n            allowance += T * max_abs_diff(E, S, (double[3]){0, 0, 0}, 0.0);\n"
     "            flags++;\n            kinds |= kind;\n            px->count_slack++;",
     "/* the other side might drop it */\n            allowance += T * max_abs_diff(E, S, (double[3]){0, 0, 0}, 0.0);\n"
     "            flags++;\n            kinds |= kind;\n            px->count_slack += 2;"),
    ("ert_margin_x100", "if (A - sc->ert_threshold < sc->ert_margin) {",
     "if (A - sc->ert_threshold < 100.0 * sc->ert_margin) {"),
    ("ert_before_margin_x100", "if (sc->ert_threshold - A < sc->ert_margin) {",
     "if (sc->ert_threshold - A < 100.0 * sc->ert_margin) {"),
    ("ert_allowance_is_A",
     "/* the other side might go on */\n                allowance += 1.0 - A;",
     "/* the other side might go on */\n                allowance += A;"),
    ("iso_margin_x100", "return m + P->sc->iso_margin * (1.0 + fabs(x));",
     "return m + 100.0 * P->sc->iso_margin * (1.0 + fabs(x));"),
    ("iso_always_unconstrained", "    if (unconstrained) {\n        px->allowance = 2.0;",
     "    if (1) {\n        px->allowance = 2.0;"),
    ("iso_unconstrained_by_any_flag", "    if (unconstrained) {\n        px->allowance = 2.0;",
     "    if (px->flags) {\n        px->allowance = 2.0;"),
    ("iso_crossing_flag_ignored", "if (flagged_here || prev_flagged) unconstrained = 1;",
     "if (flagged_here) unconstrained = 1;"),
    ("iso_pending_ignored", "if (pending && sides != pending_sides) unconstrained = 1;", ""),
    ("iso_margin_without_position", "        m += up > dn ? up : dn;\n", ""),
    ("iso_margin_one_side", "m += up > dn ? up : dn;", "m += up;"),
]

CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, pins
lib = oracle.load({lib!r})
for pin in pins.ALL_PINS:
    try:
        pin(lib)
    except (AssertionError, ValueError) as e:
        print("CAUGHT", pin.__name__)
        sys.exit(0)
print("SURVIVED")
sys.exit(3)
"""


def _run_mutant(tmp, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, f"mutation site of {name} not unique/absent"
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(find, repl))
    lib = os.path.join(tmp, f"lib{name}.so")
    subprocess.run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "oracle"), "-o", lib, path, "-lm"], check=True)
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    return name, p.returncode, (p.stdout + p.stderr)[-400:]


@pytest.mark.slow
def test_every_mutant_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=max(1, min(6, os.cpu_count() or 1))) as ex:
            results = list(ex.map(lambda m: _run_mutant(tmp, *m), MUTANTS))
    survived = [(n, out) for n, rc, out in results if rc == 3]
    assert not survived, "mutants not caught by any pin: " + "; ".join(n for n, _ in survived)


def test_mutation_sites_exist():
    src = open(SRC).read()
    for name, find, _ in MUTANTS:
        assert src.count(find) == 1, name
