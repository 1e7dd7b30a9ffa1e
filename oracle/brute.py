"""Pure-Python per-sample ray caster for tiny grids (test infrastructure only).

An independent second implementation of the same method as isaac_oracle.c,
written without looking at memory layouts: it reads each source through its
logical value array [z+g][y+g][x+g][c] instead of byte pointers and strides,
parses functor chains with a regular expression instead of a hand scanner,
and uses Python floats (IEEE binary64) throughout.  On 8^3 scenes it must
agree with the C oracle to 1e-12, which pins the C oracle's addressing,
parsing and loop structure.

Method (Matthes et al., ISAAC): one ray per pixel (Sec. 3.1); at each scan
point every enabled source is read at integer indices, passed through its
functor chain (Sec. 3.3, Tab. "functors"), interpolated or taken from the
nearest cell, classified by its transfer function and combined into one
colour and opacity, then composited front to back (Sec. 3.2).
"""

from __future__ import annotations

import math
import re

_FUNCTOR = re.compile(r"^\s*(add|mul|pow|length|sum)\s*(?:\(\s*([^)]*?)\s*\))?\s*$")


def parse_chain(text, f_dim):
    """List of (name, args); raises ValueError for an invalid chain."""
    ops = []
    if text is None or text.strip() == "":
        return ops
    dim = f_dim
    for part in text.split("|"):
        m = _FUNCTOR.match(part)
        if not m:
            raise ValueError(f"bad functor {part!r}")
        name, arg_text = m.group(1), m.group(2)
        args = [] if arg_text in (None, "") else [float(a) for a in arg_text.split(",")]
        if name in ("add", "mul", "pow"):
            if len(args) not in (1, dim):
                raise ValueError(f"{name} takes 1 or {dim} arguments")
            ops.append((name, args))
        else:
            if args:
                raise ValueError(f"{name} takes no arguments")
            ops.append((name, []))
            dim = 1
    if len(ops) > 8:
        raise ValueError("too many functors")
    return ops


def apply_chain(ops, vec):
    v = list(vec)
    for name, args in ops:
        if name in ("add", "mul", "pow"):
            a = args * len(v) if len(args) == 1 else args
            if name == "add":
                v = [x + y for x, y in zip(v, a)]
            elif name == "mul":
                v = [x * y for x, y in zip(v, a)]
            else:
                v = [_pow(x, y) for x, y in zip(v, a)]
        elif name == "length":
            v = [math.sqrt(sum(x * x for x in v))]
        else:
            v = [sum(v)]
    return v[0]


def _pow(x, y):
    """IEEE pow: a negative base with a non-integer exponent is NaN."""
    if math.isnan(x) or math.isnan(y):
        return 1.0 if y == 0.0 else math.nan
    try:
        return math.pow(x, y)
    except ValueError:
        return math.nan
    except OverflowError:
        return math.inf


def pl(points, x):
    """Piecewise-linear RGBA through (x, r, g, b, a) control points."""
    for k in range(len(points) - 1):
        x0, x1 = points[k][0], points[k + 1][0]
        if x <= x1 or k == len(points) - 2:
            w = (x - x0) / (x1 - x0)
            return [points[k][1 + c] + w * (points[k + 1][1 + c] - points[k][1 + c]) for c in range(4)]
    raise AssertionError


def classify(table, x):
    t = 0.0 if math.isnan(x) else min(max(x, 0.0), 1.0)
    u = 255.0 * t
    j = min(int(math.floor(u)), 254)
    f = u - j
    return [table[j][c] + f * (table[j + 1][c] - table[j][c]) for c in range(4)]


def _sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _norm(v):
    n = math.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
    return [v[0] / n, v[1] / n, v[2] / n]


def render(scene):
    """Returns (image[h][w][4] as nested lists, samples[h][w])."""
    out = render_flagged(scene, None, None)
    return out["image"], out["samples"]


def _nearest_alternatives(p, dims, delta):
    """Cells and flagged axes of the nearest-cell decision at p: per axis the cell
    floor(p) (clamped) and, when p lies closer than delta to an interior cell
    boundary b (1 <= b <= n-1), the cell on the other side of b."""
    cell, other = [], []
    for a in range(3):
        c = min(max(int(math.floor(p[a])), 0), dims[a] - 1)
        cell.append(c)
        b = int(math.floor(p[a] + 0.5))            # the boundary nearest to p
        if 1 <= b <= dims[a] - 1 and abs(p[a] - b) < delta:
            other.append((a, b - 1 if c == b else b))
    return cell, other


def render_flagged(scene, delta, ert_margin):
    """The ray caster with the decision bookkeeping of the several-correct-results
    reading: a decision taken within `delta` voxels of a clip plane (distance
    |n.p + d| / |n|), of the box exit (|t1 - t| along the ray) or of an interior
    nearest-cell boundary, or with an opacity within `ert_margin` of the
    termination threshold, may go the other way; each such decision adds to the
    pixel's allowance the most it can change the result.  A scan point kept or
    dropped near a plane or the exit changes the composite by its own
    contribution T (|E|max + S), T the transmittance in front of it, and the
    sample count by one; a nearest cell near a boundary by T times the largest
    change (|dE|max + |dS|) over the alternative cells; stopping or going on at
    the threshold by 1 - A.  delta=None: no bookkeeping (plain render).

    Returns dict(image, samples, allowance, flags, count_slack) as nested lists."""
    cam = scene.camera
    nx, ny, nz = scene.dims
    dims = (nx, ny, nz)
    fwd = _norm(_sub(cam.center, cam.eye))
    right = _norm(_cross(fwd, cam.up))
    upp = _cross(right, fwd)
    ortho = cam.projection == "orthographic"
    h = 0.5 * cam.ortho_height if ortho else math.tan(0.5 * cam.fovy_deg * math.pi / 180.0)
    W, H = scene.width, scene.height
    aspect = W / H
    srcs = []
    for s in scene.sources:
        table = [pl(s.tf, j / 255.0) for j in range(256)]
        srcs.append((s, parse_chain(s.chain, s.f_dim), table))
    bookkeeping = delta is not None

    def value(s, ops, x, y, z):
        g = s.guard
        return apply_chain(ops, [float(s.values[z + g, y + g, x + g, c]) for c in range(s.f_dim)])

    def point(p, cell=None):
        """Mixed premultiplied colour E and opacity S at p (cell overrides the nearest cell)."""
        S, E = 0.0, [0.0, 0.0, 0.0]
        for s, ops, table in srcs:
            if not s.enabled:
                continue
            if scene.interpolation == 0:
                q = cell if cell is not None else [min(max(int(math.floor(p[a])), 0), dims[a] - 1)
                                                   for a in range(3)]
                val = value(s, ops, *q)
            else:
                u = [p[a] - 0.5 for a in range(3)]
                i0 = [int(math.floor(u[a])) for a in range(3)]
                f = [u[a] - i0[a] for a in range(3)]
                val = 0.0
                for cz in (0, 1):
                    for cy in (0, 1):
                        for cx in (0, 1):
                            q = [i0[0] + cx, i0[1] + cy, i0[2] + cz]
                            if s.guard < 1:
                                q = [min(max(q[a], 0), dims[a] - 1) for a in range(3)]
                            w = ((f[0] if cx else 1.0 - f[0]) * (f[1] if cy else 1.0 - f[1])
                                 * (f[2] if cz else 1.0 - f[2]))
                            val += w * value(s, ops, *q)
            r, g, b, al = classify(table, val)
            wa = s.weight * al
            S += wa
            E = [E[0] + wa * r, E[1] + wa * g, E[2] + wa * b]
        if S > 1.0:
            E = [e / S for e in E]
            S = 1.0
        return E, S

    def change(E, S, E2, S2):
        return max(abs(E[c] - E2[c]) for c in range(3)) + abs(S - S2)

    img = [[[0.0] * 4 for _ in range(W)] for _ in range(H)]
    cnt = [[0] * W for _ in range(H)]
    allow = [[0.0] * W for _ in range(H)]
    nflags = [[0] * W for _ in range(H)]
    slack = [[0] * W for _ in range(H)]
    for j in range(H):
        for i in range(W):
            x = (2.0 * (i + 0.5) / W - 1.0) * h * aspect
            y = (1.0 - 2.0 * (j + 0.5) / H) * h
            if ortho:
                o = [cam.eye[a] + x * right[a] + y * upp[a] for a in range(3)]
                d = list(fwd)
            else:
                o = list(cam.eye)
                d = _norm([fwd[a] + x * right[a] + y * upp[a] for a in range(3)])
            t0, t1, hit = -math.inf, math.inf, True
            for a in range(3):
                if d[a] == 0.0:
                    if not (0.0 <= o[a] <= dims[a]):
                        hit = False
                    continue
                ta, tb = (0.0 - o[a]) / d[a], (dims[a] - o[a]) / d[a]
                t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
            t0 = max(t0, 0.0)
            if not hit or not t1 > t0:
                continue
            C, A, n, k = [0.0, 0.0, 0.0], 0.0, 0, 0
            al, nf, sl = 0.0, 0, 0
            while True:
                t = t0 + (k + 0.5) * scene.step
                k += 1
                inside = t < t1
                # a point just past the exit is only looked at for the bookkeeping
                if not inside and not (bookkeeping and t - t1 < delta):
                    break
                p = [o[a] + t * d[a] for a in range(3)]
                clipped = any(pc[0] * p[0] + pc[1] * p[1] + pc[2] * p[2] + pc[3] < 0.0 for pc in scene.clip)
                keep = inside and not clipped
                near = False
                if bookkeeping:
                    near = abs(t1 - t) < delta or any(
                        abs(pc[0] * p[0] + pc[1] * p[1] + pc[2] * p[2] + pc[3])
                        < delta * math.sqrt(pc[0] ** 2 + pc[1] ** 2 + pc[2] ** 2) for pc in scene.clip)
                if not keep:
                    if near:                         # kept on the other side
                        E, S = point(p)
                        al += (1.0 - A) * (max(abs(e) for e in E) + abs(S))
                        nf += 1
                        sl += 1
                    if not inside:
                        break
                    continue
                E, S = point(p)
                if near:                             # dropped on the other side
                    al += (1.0 - A) * (max(abs(e) for e in E) + abs(S))
                    nf += 1
                    sl += 1
                if bookkeeping and scene.interpolation == 0:
                    cell, other = _nearest_alternatives(p, dims, delta)
                    if other:
                        worst = 0.0
                        for mask in range(1, 1 << len(other)):
                            q = list(cell)
                            for b, (a, c2) in enumerate(other):
                                if mask >> b & 1:
                                    q[a] = c2
                            E2, S2 = point(p, q)
                            worst = max(worst, change(E, S, E2, S2))
                        al += (1.0 - A) * worst
                        nf += 1
                C = [C[c] + (1.0 - A) * E[c] for c in range(3)]
                A = A + (1.0 - A) * S
                n += 1
                if A >= scene.ert_threshold:
                    if bookkeeping and A - scene.ert_threshold < ert_margin:   # might go on
                        al += 1.0 - A
                        nf += 1
                    break
                if bookkeeping and scene.ert_threshold - A < ert_margin:        # might stop here
                    al += 1.0 - A
                    nf += 1
            img[j][i] = [C[0], C[1], C[2], A]
            cnt[j][i] = n
            allow[j][i], nflags[j][i], slack[j][i] = al, nf, sl
    return dict(image=img, samples=cnt, allowance=allow, flags=nflags, count_slack=slack)
