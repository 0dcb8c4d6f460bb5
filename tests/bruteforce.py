"""Exact brute-force renderer for tiny inputs (pure Python integers/fractions).

It pins the oracle with formulations of its own rather than re-typing the
oracle's formulas:

* float32 arithmetic of the vertex stage is emulated exactly: every operation
  is carried out on rationals and rounded once to the nearest float32 (ties to
  even), i.e. the IEEE-754 definition, not the host FPU;
* coverage is a strict point-in-triangle test, by Cramer's rule, of the pixel
  sample moved by (+2^-40, -2^-80) -- a concrete instance of the symbolic
  perturbation that defines a top-left fill rule in y-up coordinates.  The
  perturbed point can never lie on an edge of a non-degenerate triangle whose
  fixed-point coordinates stay below 2^24, so the strict test always decides;
* depth and perspective-correct barycentrics are exact rationals.

Every pixel is tested against every triangle whose (generously padded)
bounding box contains it, so the result does not depend on any bbox formula.
"""
from __future__ import annotations

from fractions import Fraction as F
import math

import numpy as np

EPS_X = F(1, 1 << 40)
EPS_Y = F(1, 1 << 80)


def round_f32(q: F) -> F:
    """Nearest float32 to the rational q (ties to even); +-inf on overflow."""
    if q == 0:
        return F(0)
    sign = -1 if q < 0 else 1
    a = -q if q < 0 else q
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while F(2) ** e > a:
        e -= 1
    while F(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)                        # subnormal range keeps a fixed quantum
    quantum = F(2) ** (e - 23)
    m = round(a / quantum)                  # Fraction.__round__ is half-to-even
    r = m * quantum
    if r >= F(2) ** 128 - F(2) ** 103:      # rounds past the largest finite float32
        return F(sign) * F(10) ** 60        # stand-in for infinity (fails every test below)
    return sign * r


def f32(x) -> F:
    """Exact value of a float32 input."""
    return F(float(np.float32(x)))


def rint_even(q: F) -> int:
    return round(q)


class _Vtx:
    __slots__ = ("valid", "X", "Y", "z", "iw")


def vertex(x, y, z, mvp, W, H) -> _Vtx:
    """Transform, divide, viewport and snap of one vertex, every float32
    operation rounded exactly once."""
    x, y, z = f32(x), f32(y), f32(z)
    o = _Vtx()
    if mvp is not None:
        m = [f32(v) for v in np.asarray(mvp, np.float32).reshape(16)]
        c = []
        for r in range(4):
            t = round_f32(m[4 * r] * x)
            t = round_f32(t + round_f32(m[4 * r + 1] * y))
            t = round_f32(t + round_f32(m[4 * r + 2] * z))
            t = round_f32(t + m[4 * r + 3])
            c.append(t)
    else:
        c = [x, y, z, F(1)]
    big = F(10) ** 50
    o.valid = all(abs(v) < big for v in c) and c[3] > 0
    if not o.valid:
        return o
    iw = round_f32(F(1) / c[3])
    xn = round_f32(c[0] * iw)
    yn = round_f32(c[1] * iw)
    zn = round_f32(c[2] * iw)
    xs = round_f32(round_f32(xn + 1) * round_f32(F(W, 2)))
    ys = round_f32(round_f32(yn + 1) * round_f32(F(H, 2)))
    if not (abs(zn) < big and abs(iw) < big and abs(xs) < 16384 and abs(ys) < 16384):
        o.valid = False
        return o
    o.X = rint_even(round_f32(xs * 256))
    o.Y = rint_even(round_f32(ys * 256))
    o.z, o.iw = zn, iw
    return o


def _cramer(vx, vy, px, py):
    """Barycentric (l0, l1, l2) of point (px, py) in triangle (vx, vy), exact."""
    x0, x1, x2 = vx
    y0, y1, y2 = vy
    det = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    n1 = (px - x0) * (y2 - y0) - (x2 - x0) * (py - y0)
    n2 = (x1 - x0) * (py - y0) - (px - x0) * (y1 - y0)
    return det, n1, n2


def render(sc):
    """Brute-force render of a single scene (gouraud).  Returns dict with
    cover [H][W] (covering triangle count), winner [H][W] (-1 if none),
    zexact [H][W] (Fraction or None), color [H][W][3] (floats from exact
    rationals), cand[(py, px)] -> list of (zexact, t) of covering triangles
    with 0 <= z < 1."""
    W, H = int(sc.width), int(sc.height)
    V = sc.pos.shape[1]
    mvp = None if sc.mvp is None else np.asarray(sc.mvp).reshape(-1)[:16]
    verts = [vertex(sc.pos[0, v], sc.pos[1, v], sc.pos[2, v], mvp, W, H) for v in range(V)]
    cover = np.zeros((H, W), np.int64)
    cand = {}
    tris = []
    for t in range(int(sc.num_tris)):
        vid = [int(sc.idx[t, k]) if sc.idx is not None else 3 * t + k for k in range(3)]
        vs = [verts[v] for v in vid]
        if not all(v.valid for v in vs):
            continue
        vx = [v.X for v in vs]
        vy = [v.Y for v in vs]
        det = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0])
        if det == 0:
            continue
        tris.append((t, vid, vs))
        # generous pixel range: any sample inside lies within [min, max]
        x_lo = max(0, min(vx) // 256 - 1)
        x_hi = min(W - 1, max(vx) // 256 + 1)
        y_lo = max(0, min(vy) // 256 - 1)
        y_hi = min(H - 1, max(vy) // 256 + 1)
        # scale by 2^80 so the perturbed sample has integer coordinates
        S = 1 << 80
        VX = [x * S for x in vx]
        VY = [y * S for y in vy]
        for py in range(y_lo, y_hi + 1):
            PY = (256 * py + 128) * S - 1                      # - 2^-80 px*256 units
            for px in range(x_lo, x_hi + 1):
                PX = (256 * px + 128) * S + (1 << 40)          # + 2^-40
                d, n1, n2 = _cramer(VX, VY, PX, PY)
                if d < 0:
                    d, n1, n2 = -d, -n1, -n2
                if not (n1 > 0 and n2 > 0 and d - n1 - n2 > 0):
                    continue
                cover[py, px] += 1
                # exact depth at the unperturbed sample
                d0, m1, m2 = _cramer(vx, vy, 256 * px + 128, 256 * py + 128)
                l1, l2 = F(m1, d0), F(m2, d0)
                l0 = 1 - l1 - l2
                z = l0 * vs[0].z + l1 * vs[1].z + l2 * vs[2].z
                if 0 <= z < 1:
                    cand.setdefault((py, px), []).append((z, t, (l0, l1, l2), vid, vs))
    winner = -np.ones((H, W), np.int64)
    zex = np.empty((H, W), dtype=object)
    color = np.zeros((H, W, 3), np.float64)
    for (py, px), lst in cand.items():
        zb = [(round_f32(z), t) for (z, t, *_r) in lst]
        best = min(zb)
        i = zb.index(best)
        z, t, lam, vid, vs = lst[i]
        winner[py, px] = t
        zex[py, px] = z
        q = [lam[k] * vs[k].iw for k in range(3)]
        Q = sum(q)
        bp = [qk / Q for qk in q]
        for c in range(3):
            color[py, px, c] = float(sum(bp[k] * f32(sc.color[c, vid[k]]) for k in range(3)))
    return dict(cover=cover, winner=winner, zexact=zex, color=color, cand=cand)


def bins(sc, bin_size: int):
    """Brute-force AssignToBoundingBox from exact bboxes: for every live
    triangle, every bin whose pixel rectangle contains a pixel whose sample
    lies inside the triangle's vertex bounding box.  Returns {bin: sorted list}."""
    W, H = int(sc.width), int(sc.height)
    V = sc.pos.shape[1]
    mvp = None if sc.mvp is None else np.asarray(sc.mvp).reshape(-1)[:16]
    verts = [vertex(sc.pos[0, v], sc.pos[1, v], sc.pos[2, v], mvp, W, H) for v in range(V)]
    bw = bin_size or W
    bh = bin_size or H
    nbx = -(-W // bw)
    out = {}
    for t in range(int(sc.num_tris)):
        vid = [int(sc.idx[t, k]) if sc.idx is not None else 3 * t + k for k in range(3)]
        vs = [verts[v] for v in vid]
        if not all(v.valid for v in vs):
            continue
        vx = [v.X for v in vs]
        vy = [v.Y for v in vs]
        if (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]) == 0:
            continue
        xs = [px for px in range(W) if min(vx) <= 256 * px + 128 <= max(vx)]
        ys = [py for py in range(H) if min(vy) <= 256 * py + 128 <= max(vy)]
        if not xs or not ys:
            continue
        for by in range(ys[0] // bh, ys[-1] // bh + 1):
            for bx in range(xs[0] // bw, xs[-1] // bw + 1):
                out.setdefault(by * nbx + bx, []).append(t)
    return out
