"""Pins of the oracle's Reyes front end (Split and Dice of bicubic Bezier
patches) against what the mathematics fixes, independently of de Casteljau:

* a bicubic Bezier patch is sum_ij B_i(v) B_j(u) P_ij with the cubic
  Bernstein basis B_k(t) = C(3, k) t^k (1 - t)^(3 - k), evaluated here in
  float64 straight from that definition;
* a control net that is an affine function of (j/3, i/3) gives the affine
  surface A + u U + v V (Bezier curves reproduce linear functions), so its
  dice grid and central-difference normals have closed forms;
* halving at 1/2 must reparametrise: the lower half at s is the patch at s/2,
  the upper half the patch at 1/2 + s/2;
* an axis-aligned square of S = D 2^k pixels splits into exactly 4^k leaves
  of D pixels, and into 2^d leaves of known shape when the depth is capped.

Each check returns True when it holds; tests/test_oracle_reyes.py runs them
all, and tests/test_oracle_mutants.py runs them against planted mistakes.
"""
from math import comb

import numpy as np

import oracle


def bernstein(cp, u, v):
    """Patch point at (u, v) in float64 from the Bernstein definition."""
    P = np.asarray(cp, np.float64).reshape(4, 4, 3)
    bu = np.array([comb(3, k) * u ** k * (1 - u) ** (3 - k) for k in range(4)])
    bv = np.array([comb(3, k) * v ** k * (1 - v) ** (3 - k) for k in range(4)])
    return np.einsum("i,j,ijc->c", bv, bu, P)


def net(fn):
    """16 control points [16][3] float32 with point 4i + j = fn(j / 3, i / 3)."""
    return np.array([fn(j / 3.0, i / 3.0) for i in range(4) for j in range(4)], np.float32)


def square(x0, y0, s, z=0.5):
    """Flat patch over NDC [x0, x0 + s] x [y0, y0 + s] at depth z (u along x)."""
    return net(lambda u, v: (x0 + s * u, y0 + s * v, z))


def halves():
    rng = np.random.default_rng(3)
    cp = rng.standard_normal((16, 3)).astype(np.float32)
    ok = True
    for d in (0, 1):
        lo, hi = oracle.reyes_halve(cp, d)
        for s in (0.0, 0.3, 0.75, 1.0):
            for t in (0.0, 0.45, 1.0):
                if d == 0:
                    want_lo, want_hi = bernstein(cp, s / 2, t), bernstein(cp, 0.5 + s / 2, t)
                else:
                    want_lo, want_hi = bernstein(cp, s, t / 2), bernstein(cp, s, 0.5 + t / 2)
                ok &= np.allclose(bernstein(lo, s, t), want_lo, rtol=0, atol=2e-5)
                ok &= np.allclose(bernstein(hi, s, t), want_hi, rtol=0, atol=2e-5)
    return bool(ok)


def affine_dice():
    A, U, V = np.array([0.1, -0.2, 0.4]), np.array([0.5, 0.1, -0.2]), np.array([-0.15, 0.6, 0.25])
    cp = net(lambda u, v: A + u * U + v * V)
    n = 5
    col = np.array([[0.25, 0.5, 0.75]], np.float32)
    pos, c, nrm, idx = oracle.reyes_dice(cp[None], np.zeros(1, np.int32), col, n)
    m = n + 1
    ok = pos.shape == (3, m * m) and idx.shape == (2 * n * n, 3)
    area = 0.0
    for i in range(m):
        for j in range(m):
            k = i * m + j
            ok &= np.allclose(pos[:, k], A + (j / n) * U + (i / n) * V, rtol=0, atol=3e-7)
            du = (min(j + 1, n) - max(j - 1, 0)) / n
            dv = (min(i + 1, n) - max(i - 1, 0)) / n
            ok &= np.allclose(nrm[:, k], np.cross(du * U, dv * V), rtol=1e-5, atol=1e-7)
            ok &= bool((c[:, k] == col[0]).all())
    # triangles: counter-clockwise in (u, v), tiling the unit square
    uv = np.array([(k % m / n, k // m / n) for k in range(m * m)])
    for t in idx:
        a, b, d = uv[t[0]], uv[t[1]], uv[t[2]]
        sa = 0.5 * ((b[0] - a[0]) * (d[1] - a[1]) - (b[1] - a[1]) * (d[0] - a[0]))
        ok &= sa > 0
        area += sa
    ok &= abs(area - 1.0) < 1e-9
    edges = {}
    for t in idx:
        for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            edges[tuple(sorted(e))] = edges.get(tuple(sorted(e)), 0) + 1
    ok &= sum(1 for v in edges.values() if v == 1) == 4 * n   # the border, once each
    ok &= all(v in (1, 2) for v in edges.values())
    return bool(ok)


def surface():
    """Every diced vertex of a split height field lies on the original patch,
    and the leaves tile its parameter square exactly once."""
    rng = np.random.default_rng(5)
    zs = rng.uniform(0.3, 0.7, 16)
    x0, y0, s = -0.8, -0.7, 1.4
    cp = net(lambda u, v: (x0 + s * u, y0 + s * v, 0.0))
    cp[:, 2] = zs
    W = H = 64
    leaves, src = oracle.reyes_split(cp[None], None, W, H, 4.0, 20)
    ok = len(leaves) > 16 and bool((src == 0).all())
    area = 0.0
    for lf in leaves:
        u0, u1 = (lf[:, 0].min() - x0) / s, (lf[:, 0].max() - x0) / s
        v0, v1 = (lf[:, 1].min() - y0) / s, (lf[:, 1].max() - y0) / s
        area += (u1 - u0) * (v1 - v0)
        ok &= (u1 - u0) * s * W / 2 <= 4.0 + 1e-4 and (v1 - v0) * s * H / 2 <= 4.0 + 1e-4
    ok &= abs(area - 1.0) < 1e-5
    pos, _, _, _ = oracle.reyes_dice(leaves, src, np.ones((1, 3), np.float32), 4)
    for k in range(0, pos.shape[1], 7):
        u, v = (pos[0, k] - x0) / s, (pos[1, k] - y0) / s
        ok &= abs(pos[2, k] - bernstein(cp, u, v)[2]) < 3e-6
    return bool(ok)


def counts():
    """A 128 px square, D = 8: 4^4 leaves of 8 x 8 px; capped at depth 3:
    8 leaves of 32 x 64 px (u first on ties, then the longer direction)."""
    W = H = 256
    cp = square(-0.5, -0.5, 1.0)
    leaves, _ = oracle.reyes_split(cp[None], None, W, H, 8.0, 20)
    ok = len(leaves) == 256
    # (inner control points at thirds are not exact in binary, so a half's
    # end point may be a rounding away from the exact midpoint)
    near = lambda a, b: abs(a - b) < 1e-3  # noqa: E731
    ok &= all(near(np.ptp(lf[:, 0]) * W / 2, 8.0) and near(np.ptp(lf[:, 1]) * H / 2, 8.0)
              for lf in leaves)
    capped, _ = oracle.reyes_split(cp[None], None, W, H, 8.0, 3)
    ok &= len(capped) == 8
    ok &= all(near(np.ptp(lf[:, 0]) * W / 2, 32.0) and near(np.ptp(lf[:, 1]) * H / 2, 64.0)
              for lf in capped)
    return bool(ok)


def offscreen():
    """A 64 px square from -8 to 56 px on a 64 px screen, D = 4: 16 x 16
    cells of 4 px; the first column and row end before the screen starts
    (the second one's far edge, x = 0 or y = 0, still touches it): 15 x 15
    leaves.  Shifted to -12..52 px, two columns and rows drop: 14 x 14."""
    W = H = 64
    cp = square(-1.25, -1.25, 2.0)
    leaves, _ = oracle.reyes_split(cp[None], None, W, H, 4.0, 20)
    ok = len(leaves) == 15 * 15
    cp2 = square(-1.375, -1.375, 2.0)
    l2, _ = oracle.reyes_split(cp2[None], None, W, H, 4.0, 20)
    ok &= len(l2) == 14 * 14
    return bool(ok)


def decisions():
    D = 8.0
    ok = oracle.reyes_decide(square(-0.05, -0.05, 0.05), None, 256, 256, D) == 1   # 6.4 px
    ok &= oracle.reyes_decide(square(0.0, 0.0, 0.0625), None, 256, 256, D) == 1      # exactly 8 px
    ok &= oracle.reyes_decide(square(0.0, 0.0, 0.0626), None, 256, 256, D) == 2      # tie: u
    wide = net(lambda u, v: (0.4 * u, 0.05 * v, 0.5))
    tall = net(lambda u, v: (0.05 * u, 0.4 * v, 0.5))
    ok &= oracle.reyes_decide(wide, None, 256, 256, D) == 2
    ok &= oracle.reyes_decide(tall, None, 256, 256, D) == 3
    # the u direction running along screen y: still a split in u
    rot = net(lambda u, v: (0.05 * v, 0.4 * u, 0.5))
    ok &= oracle.reyes_decide(rot, None, 256, 256, D) == 2
    ok &= oracle.reyes_decide(square(0.0, 0.0, 0.4), None, 256, 256, D, last=True) == 1
    for shift in ((1.01, 0.0), (-1.5, 0.0), (0.0, 1.01), (0.0, -1.5)):
        ok &= oracle.reyes_decide(square(shift[0], shift[1], 0.4), None, 256, 256, D) == 0
    nan = square(0.0, 0.0, 0.4)
    nan[5, 1] = np.nan
    ok &= oracle.reyes_decide(nan, None, 256, 256, D) == 0
    # perspective: a control point behind the eye (clip w <= 0) drops the patch
    f = 1.0
    mvp = np.array([[f, 0, 0, 0], [0, f, 0, 0], [0, 0, 1, -0.1], [0, 0, 1, 0]], np.float32)
    behind = net(lambda u, v: (0.1 * u, 0.1 * v, 1.0 - 1.2 * u * v))   # w = -0.2 at (1, 1)
    ok &= oracle.reyes_decide(behind, mvp, 256, 256, D) == 0
    front = net(lambda u, v: (0.01 * u, 0.01 * v, 1.0))
    ok &= oracle.reyes_decide(front, mvp, 256, 256, D) == 1
    return bool(ok)


def bfs_order():
    """Round 0's leaves come first (in input order), then each later round's,
    lower halves before upper ones."""
    W = H = 64
    big = square(-0.5, -0.5, 0.5)      # 16 px: split u, then v -> 4 leaves of 8 px
    small = square(0.5, 0.5, 0.125)    # 4 px: a leaf at once
    leaves, src = oracle.reyes_split(np.stack([big, small]), None, W, H, 8.0, 20)
    ok = list(src) == [1, 0, 0, 0, 0]
    corners = [(float(lf[:, 0].min()), float(lf[:, 1].min())) for lf in leaves[1:]]
    ok &= corners == [(-0.5, -0.5), (-0.5, -0.25), (-0.25, -0.5), (-0.25, -0.25)]
    return bool(ok)


def end_to_end():
    """Two flat patches side by side, diced and drawn: exactly the pixels
    whose centres they cover, each with its patch's colour times n.l."""
    W, H = 64, 40
    # NDC x in [-0.5, 0] and [0, 0.5] -> px 16..32 and 32..48; y in [-0.5, 0.5] -> 10..30
    p0 = net(lambda u, v: (-0.5 + 0.5 * u, -0.5 + v, 0.5))
    p1 = net(lambda u, v: (0.5 * u, -0.5 + v, 0.5))
    from types import SimpleNamespace
    col = np.array([[0.9, 0.3, 0.2], [0.1, 0.7, 0.4]], np.float32)
    ps = SimpleNamespace(width=W, height=H, patches=np.stack([p0, p1]), patch_color=col, mvp=None,
                         dice_px=4.0, max_depth=20, dice_n=3,
                         lights=np.array([[0.0, 0.6, 0.8]], np.float32))
    sc = oracle.reyes_scene(ps)
    o = oracle.render(sc)
    pid = o["primid"][0]
    inside = np.zeros((H, W), bool)
    inside[10:30, 16:48] = True
    ok = bool(((pid >= 0) == inside).all())
    img = o["color"][0, :, :, :3]
    ok &= np.allclose(img[10:30, 16:32], col[0] * np.float32(0.8), rtol=1e-6, atol=0)
    ok &= np.allclose(img[10:30, 32:48], col[1] * np.float32(0.8), rtol=1e-6, atol=0)
    ok &= sc.num_tris == 2 * 9 * sc.num_leaves
    return bool(ok)


PINS = {"halves": halves, "affine_dice": affine_dice, "surface": surface, "counts": counts,
        "offscreen": offscreen, "decisions": decisions, "bfs_order": bfs_order,
        "end_to_end": end_to_end}
