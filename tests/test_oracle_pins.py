"""Pins of the CPU oracle against facts that do not come from the oracle.

The oracle is the plain definition of the image (for every pixel sample, the
nearest covering triangle; Piko Sec. 4.1 phases, Sec. 7.1 rasterizer stages).
Here it is checked against: an exact brute force that formulates coverage and
depth differently; closed forms (rectangle areas, watertight partitions, fans
around a sample-centred vertex, lattice-translation averages); special cases
(constant depth, vertex-coincident samples, texel centres, light-aligned
normals); hand-worked snap values; and central finite differences, which are
exact for the quadratic image loss.
"""
import math
import os
from types import SimpleNamespace

import numpy as np
import pytest

import bruteforce as bf
import oracle
from paper_1404_6293_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cross2(a, b):
    return int(a[0]) * int(b[1]) - int(a[1]) * int(b[0])


def ulp32(x: float) -> float:
    x = np.float32(abs(x))
    return float(np.spacing(x)) if x != 0 else float(np.spacing(np.float32(0)))


def _ndc_scene(W, H, X, Y, Z, color=None, idx=None, **kw):
    """A scene whose vertices sit exactly on chosen fixed-point positions:
    x_ndc = X/(128 W) - 1 is exact in float32 for the sizes used here, so the
    snap returns X unchanged (checked separately by test_lattice_roundtrip)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    pos = np.stack([X / (128.0 * W) - 1.0, Y / (128.0 * H) - 1.0, np.asarray(Z, np.float64)])
    pos = pos.astype(np.float32)
    V = pos.shape[1]
    if color is None:
        color = np.random.default_rng(0).uniform(0, 1, (3, V)).astype(np.float32)
    T = (V // 3) if idx is None else len(idx)
    d = dict(width=W, height=H, pos=pos, color=np.asarray(color, np.float32),
             idx=None if idx is None else np.asarray(idx, np.int32), num_tris=T, mvp=None,
             num_scenes=1, scene_tri_off=None, scene_vtx_off=None, instanced=False, uv=None,
             normal=None, texture=None, lights=None, shading="gouraud")
    d.update(kw)
    return SimpleNamespace(**d)


# ---------------------------------------------------------------------------
# vertex stage
# ---------------------------------------------------------------------------
def test_golden_snap_cases():
    rows = []
    with open(os.path.join(GOLDEN, "snap.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("|")
            rows.append(([float(v) for v in lhs.split()], [float(v) for v in rhs.split()]))
    assert len(rows) >= 12
    for (W, H, x, y, z, w), (X, Y, valid, iw) in rows:
        mvp = np.diag([1.0, 1.0, 1.0, w]).astype(np.float32)
        sc = SimpleNamespace(width=int(W), height=int(H), pos=np.array([[x], [y], [z]], np.float32),
                             color=np.zeros((3, 1), np.float32), idx=None, num_tris=0,
                             mvp=mvp.reshape(16), uv=None, normal=None, texture=None,
                             lights=None, shading="gouraud")
        oX, oY, oz, oiw, ovalid = oracle.vertices(sc)
        assert bool(ovalid[0]) == bool(valid), (W, H, x, y, z, w)
        if valid:
            assert (oX[0], oY[0]) == (int(X), int(Y)), (W, H, x, y, z, w)
            assert oiw[0] == np.float32(iw)
            assert oz[0] == np.float32(z / w)


def test_lattice_roundtrip():
    """Fixed-point positions placed exactly in NDC come back unchanged."""
    rng = np.random.default_rng(7)
    for W, H in [(64, 64), (48, 40), (256, 256)]:
        X = rng.integers(0, 256 * W, 500)
        Y = rng.integers(0, 256 * H, 500)
        sc = _ndc_scene(W, H, X, Y, np.full(500, 0.5))
        oX, oY, _, oiw, valid = oracle.vertices(sc)
        assert valid.all()
        np.testing.assert_array_equal(oX, X)
        np.testing.assert_array_equal(oY, Y)
        assert (oiw == 1.0).all()


def test_vertex_stage_vs_exact_float32_emulation():
    """Random NDC vertices and a perspective camera: the oracle's snap equals
    the exact IEEE-float32 emulation of the same operations."""
    sc = scenes.grid(seed=11, width=40, height=24, nx=8, ny=4)
    oX, oY, oz, oiw, valid = oracle.vertices(sc)
    mvp = sc.mvp.reshape(16)
    for v in range(sc.pos.shape[1]):
        e = bf.vertex(sc.pos[0, v], sc.pos[1, v], sc.pos[2, v], mvp, sc.width, sc.height)
        assert e.valid == bool(valid[v])
        if e.valid:
            assert (oX[v], oY[v]) == (e.X, e.Y)
            assert oz[v] == float(e.z) and oiw[v] == float(e.iw)


# ---------------------------------------------------------------------------
# coverage, depth, winner and Gouraud colour against the exact brute force
# ---------------------------------------------------------------------------
def _check_against_bruteforce(sc):
    o = oracle.render(sc, want_cover=True)
    b = bf.render(sc)
    np.testing.assert_array_equal(o["cover_count"][0], b["cover"])
    assert int(o["frag_count"][0]) == int(b["cover"].sum())
    pid, dep, col = o["primid"][0], o["depth"][0], o["color"][0]
    H, W = pid.shape
    for py in range(H):
        for px in range(W):
            lst = b["cand"].get((py, px), [])
            if not lst:
                assert pid[py, px] == -1 and dep[py, px] == 1.0
                assert (col[py, px] == 0).all()
                continue
            t = int(pid[py, px])
            # the oracle's winner covers the sample, and its depth is the
            # exact rational depth within one float32 ulp
            zt = [z for (z, tt, *_r) in lst if tt == t]
            assert zt, (py, px, t)
            zt = float(zt[0])
            assert abs(dep[py, px] - zt) <= ulp32(zt), (py, px)
            # no covering triangle is nearer by more than rounding can explain
            zmin = min(float(z) for (z, *_r) in lst)
            assert zt - zmin <= 2 * ulp32(zmin), (py, px)
            if t != b["winner"][py, px]:
                zb = float(b["zexact"][py, px])
                assert abs(zt - zb) <= 2 * ulp32(zb), (py, px)
                continue
            np.testing.assert_allclose(col[py, px, :3], b["color"][py, px], rtol=1e-5, atol=1e-6)
            assert col[py, px, 3] == 1.0


@pytest.mark.parametrize("seed", range(100))
def test_small_random_vs_bruteforce(seed):
    # ragged 28x20 screen, 10 triangles of mixed size and winding
    _check_against_bruteforce(scenes.tiny(seed=seed, width=28, height=20, num_tris=10))


@pytest.mark.parametrize("seed", [1001, 5])
def test_tiny64_vs_bruteforce(seed):
    _check_against_bruteforce(scenes.tiny(seed=seed))


def test_perspective_grid_vs_bruteforce():
    """Shared vertices, an index buffer and w != 1 (perspective-correct colour)."""
    _check_against_bruteforce(scenes.grid(seed=3, width=40, height=24, nx=8, ny=4))


def test_tie_break_smaller_primid_wins():
    """Depth quantised to 4 levels with constant depth per triangle: depths are
    exact, so the winner is the smallest index among the covering triangles
    at the smallest depth."""
    rng = np.random.default_rng(12)
    W = H = 32
    T = 60
    X = rng.integers(0, 256 * W, 3 * T)
    Y = rng.integers(0, 256 * H, 3 * T)
    Z = np.repeat(rng.integers(0, 4, T) / 4.0, 3)
    sc = _ndc_scene(W, H, X, Y, Z)
    o = oracle.render(sc)
    b = bf.render(sc)
    ties = 0
    for (py, px), lst in b["cand"].items():
        zmin = min(z for (z, *_r) in lst)
        best = min(t for (z, t, *_r) in lst if z == zmin)
        ties += sum(1 for (z, *_r) in lst if z == zmin) > 1
        assert o["primid"][0, py, px] == best
        assert o["depth"][0, py, px] == float(zmin)
    assert ties > 50


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
def _jittered_partition(rng, W, H, x0, x1, y0, y1, nx, ny):
    """Triangulate the pixel-aligned rectangle [x0,x1]x[y0,y1] (pixels) with a
    jittered nx x ny grid: boundary vertices stay on the rectangle's edges,
    interior ones are jittered and some are put exactly on sample centres;
    random diagonals and random vertex order (both windings)."""
    gx = np.linspace(256 * x0, 256 * x1, nx + 1).round().astype(np.int64)
    gy = np.linspace(256 * y0, 256 * y1, ny + 1).round().astype(np.int64)
    GX, GY = np.meshgrid(gx, gy)
    step = min(gx[1] - gx[0], gy[1] - gy[0])
    J = step // 3
    inner = (slice(1, ny), slice(1, nx))
    GX[inner] += rng.integers(-J, J + 1, GX[inner].shape)
    GY[inner] += rng.integers(-J, J + 1, GY[inner].shape)
    # snap about a third of the interior vertices onto sample centres
    m = rng.uniform(size=GX[inner].shape) < 0.35
    GX[inner] = np.where(m, (GX[inner] // 256) * 256 + 128, GX[inner])
    GY[inner] = np.where(m, (GY[inner] // 256) * 256 + 128, GY[inner])
    vid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            pair = [(a, b, c), (a, c, d)] if rng.uniform() < 0.5 else [(a, b, d), (b, c, d)]
            for t in pair:
                t = list(t)
                if rng.uniform() < 0.5:
                    t = [t[0], t[2], t[1]]
                k = rng.integers(3)
                tris.append(t[k:] + t[:k])
    return GX.ravel(), GY.ravel(), np.asarray(tris, np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_watertight_partition(seed):
    """Every sample inside a triangulated pixel-aligned rectangle is covered
    exactly once; none outside (shared edges and vertices included)."""
    rng = np.random.default_rng(100 + seed)
    W, H = 48, 40
    x0, x1, y0, y1 = 3, 45, 2, 37
    X, Y, idx = _jittered_partition(rng, W, H, x0, x1, y0, y1, nx=11, ny=9)
    sc = _ndc_scene(W, H, X, Y, np.full(X.size, 0.5), idx=idx)
    o = oracle.render(sc, want_cover=True)
    cnt = o["cover_count"][0]
    inside = np.zeros((H, W), bool)
    inside[y0:y1, x0:x1] = True
    assert (cnt[inside] == 1).all()
    assert (cnt[~inside] == 0).all()
    assert int(o["frag_count"][0]) == (x1 - x0) * (y1 - y0)


@pytest.mark.parametrize("k", [3, 5, 7, 12])
def test_fan_around_sample_centre(k):
    """k triangles sharing a vertex exactly on a sample centre: that sample and
    every sample strictly inside the fan's polygon are covered exactly once."""
    rng = np.random.default_rng(k)
    W = H = 32
    cx, cy = 256 * 16 + 128, 256 * 15 + 128
    ang = np.sort(rng.uniform(0, 2 * math.pi, k))
    ang = ang + np.linspace(0, 2 * math.pi, k, endpoint=False) - ang  # spread out
    ang += rng.uniform(0, 0.3)
    r = 256 * 9
    PX = (cx + r * np.cos(ang)).round().astype(np.int64)
    PY = (cy + r * np.sin(ang)).round().astype(np.int64)
    X = np.concatenate([[cx], PX])
    Y = np.concatenate([[cy], PY])
    idx = []
    for i in range(k):
        t = [0, 1 + i, 1 + (i + 1) % k]
        if rng.uniform() < 0.5:
            t = [t[0], t[2], t[1]]
        idx.append(t)
    sc = _ndc_scene(W, H, X, Y, np.full(X.size, 0.25), idx=idx)
    o = oracle.render(sc, want_cover=True)
    cnt = o["cover_count"][0]
    assert cnt.max() <= 1
    assert cnt[15, 16] == 1
    # samples strictly inside the outer polygon (exact integer test)
    for py in range(H):
        for px in range(W):
            sx, sy = 256 * px + 128, 256 * py + 128
            inside = True
            for i in range(k):
                ax, ay, bx, by = PX[i], PY[i], PX[(i + 1) % k], PY[(i + 1) % k]
                if (bx - ax) * (sy - ay) - (by - ay) * (sx - ax) <= 0:
                    inside = False
                    break
            if inside:
                assert cnt[py, px] == 1, (py, px)


@pytest.mark.parametrize("rect", [(0, 0, 1, 1), (2, 3, 9, 4), (5, 1, 6, 30), (0, 0, 32, 32), (7, 9, 20, 26)])
def test_rectangle_count_equals_area(rect):
    x0, y0, x1, y1 = rect
    W = H = 32
    X = [256 * x0, 256 * x1, 256 * x1, 256 * x0]
    Y = [256 * y0, 256 * y0, 256 * y1, 256 * y1]
    sc = _ndc_scene(W, H, X, Y, [0.5] * 4, idx=[[0, 1, 2], [0, 2, 3]])
    o = oracle.render(sc, want_cover=True)
    assert int(o["frag_count"][0]) == (x1 - x0) * (y1 - y0)
    assert o["cover_count"][0].max() == 1


@pytest.mark.parametrize("seed", range(3))
def test_translation_average_equals_area(seed):
    """The covered-sample count of one triangle averaged over random
    sub-pixel translations approaches its area: |mean - A| within
    4 sigma/sqrt(K) + perimeter/256."""
    rng = np.random.default_rng(seed)
    cell, n = 12, 32                      # n x n copies in 12-px cells
    W = H = cell * n
    tri = rng.integers(256 * 1, 256 * (cell - 1), size=(3, 2))
    while abs(_cross2(tri[1] - tri[0], tri[2] - tri[0])) < 256 * 256 * 4:
        tri = rng.integers(256 * 1, 256 * (cell - 1), size=(3, 2))
    X, Y = [], []
    for j in range(n):
        for i in range(n):
            dx, dy = rng.integers(0, 256, 2)
            for k in range(3):
                X.append(tri[k, 0] + dx + 256 * cell * i)
                Y.append(tri[k, 1] + dy + 256 * cell * j)
    sc = _ndc_scene(W, H, X, Y, [0.5] * len(X))
    o = oracle.render(sc, want_cover=True)
    cnt = o["cover_count"][0].reshape(n, cell, n, cell).sum(axis=(1, 3)).ravel()
    A = abs(_cross2(tri[1] - tri[0], tri[2] - tri[0])) / 2 / 65536.0
    per = sum(np.hypot(*(tri[(k + 1) % 3] - tri[k])) for k in range(3)) / 256.0
    K = cnt.size
    tol = 4 * cnt.std() / math.sqrt(K) + per / 256.0
    assert abs(cnt.mean() - A) <= tol, (cnt.mean(), A, tol)


def test_constant_depth_is_exact():
    rng = np.random.default_rng(3)
    W = H = 32
    T = 40
    X = rng.integers(0, 256 * W, 3 * T)
    Y = rng.integers(0, 256 * H, 3 * T)
    zt = rng.uniform(0, 1, T).astype(np.float32)
    sc = _ndc_scene(W, H, X, Y, np.repeat(zt, 3))
    o = oracle.render(sc)
    pid, dep = o["primid"][0], o["depth"][0]
    m = pid >= 0
    assert m.sum() > 100
    np.testing.assert_array_equal(dep[m], zt[pid[m]])


def test_vertex_coincident_sample_takes_vertex_colour():
    """A vertex exactly on a sample centre: the fill rule gives that sample to
    the triangle that contains the direction just right of (and a hair below)
    the vertex; there the barycentrics are (1, 0, 0), so the colour equals the
    vertex colour exactly, for either winding and for w != 1."""
    W = H = 16
    sx, sy = 256 * 4 + 128, 256 * 6 + 128
    col = np.array([[0.25, 0.9, 0.1], [0.5, 0.3, 0.7], [0.125, 0.6, 0.2]], np.float32)
    right = ([sx, sx + 2560, sx + 2048], [sy, sy - 768, sy + 1280])   # opens to +x
    left = ([sx, sx - 2560, sx - 2048], [sy, sy + 768, sy - 1280])    # opens to -x
    for (X, Y), owns in [(right, True), (left, False)]:
        for order in ([0, 1, 2], [0, 2, 1]):
            Xo, Yo = [X[k] for k in order], [Y[k] for k in order]
            c = col[:, order]
            sc = _ndc_scene(W, H, Xo, Yo, [0.5] * 3, color=c)
            o = oracle.render(sc, want_cover=True)
            assert o["cover_count"][0, 6, 4] == int(owns)
            if owns:
                np.testing.assert_array_equal(o["color"][0, 6, 4, :3], col[:, 0])
    # the same through a perspective matrix (w = 2 at every vertex)
    sc = _ndc_scene(W, H, right[0], right[1], [0.5] * 3, color=col)
    sc.pos = (sc.pos * np.float32(2.0)).astype(np.float32)
    sc.mvp = np.diag([1.0, 1.0, 1.0, 2.0]).astype(np.float32).reshape(16)
    o = oracle.render(sc, want_cover=True)
    assert o["cover_count"][0, 6, 4] == 1
    np.testing.assert_array_equal(o["color"][0, 6, 4, :3], col[:, 0])


def test_full_grid_covers_every_pixel_once():
    """The 1024x512-quad grid through the 1920x1080 perspective camera is
    fold-free and overfills the screen: every pixel is covered exactly once."""
    sc = scenes.grid()
    live, bbox, A2 = oracle.setup(sc)
    # fold-free: every triangle keeps its counter-clockwise winding on screen;
    # the ones that fall wholly outside the screen (overfill) are culled
    assert (A2 > 0).all() and 0.7 < live.mean() < 0.9
    o = oracle.render(sc, want_bary=False, want_cover=True)
    assert (o["cover_count"][0] == 1).all()
    assert int(o["frag_count"][0]) == 1920 * 1080
    assert (o["primid"][0] >= 0).all()


# ---------------------------------------------------------------------------
# texture and deferred shading special cases
# ---------------------------------------------------------------------------
def _textured(sc, tex, uv):
    d = dict(vars(sc))
    d.update(texture=np.asarray(tex, np.float32), uv=np.asarray(uv, np.float32), shading="textured")
    return SimpleNamespace(**d)


def test_constant_texture_modulates_by_constant():
    sc = scenes.grid(seed=5, width=40, height=24, nx=8, ny=4)
    V = sc.pos.shape[1]
    uv = np.random.default_rng(1).uniform(-0.2, 1.2, (2, V))
    base = oracle.render(sc)
    tex = np.empty((5, 7, 3), np.float32)
    tex[...] = np.array([0.5, 0.25, 2.0], np.float32)
    o = oracle.render(_textured(sc, tex, uv))
    np.testing.assert_array_equal(o["primid"], base["primid"])
    np.testing.assert_allclose(o["color"][..., :3], base["color"][..., :3] * tex[0, 0],
                               rtol=3e-7, atol=1e-7)


def test_texel_centre_returns_texel():
    """A constant uv at the centre of texel (i, j) samples that texel alone
    (half-texel offsets or a transposed texture would be off by far more)."""
    rng = np.random.default_rng(4)
    tex = rng.uniform(0, 1, (6, 8, 3)).astype(np.float32)
    W = H = 16
    X = [0, 256 * 16, 0, 256 * 16]
    Y = [0, 0, 256 * 16, 256 * 16]
    for (i, j) in [(0, 0), (3, 2), (7, 5), (5, 4)]:
        u, v = (i + 0.5) / 8, (j + 0.5) / 6
        uv = np.array([[u] * 4, [v] * 4])
        col = np.ones((3, 4), np.float32)
        sc = _ndc_scene(W, H, X, Y, [0.5] * 4, color=col, idx=[[0, 1, 3], [0, 3, 2]])
        o = oracle.render(_textured(sc, tex, uv))
        # the interpolated uv can differ from the constant by an ulp (the
        # perspective weights sum to one only up to rounding), which leaks a
        # weight of ~1e-7 onto a neighbouring texel
        np.testing.assert_allclose(o["color"][0, :, :, :3],
                                   np.broadcast_to(tex[j, i], (H, W, 3)), rtol=0, atol=1e-6)


def test_deferred_light_aligned_and_orthogonal():
    W = H = 16
    X = [0, 256 * 16, 0, 256 * 16]
    Y = [0, 0, 256 * 16, 256 * 16]
    col = np.random.default_rng(2).uniform(0, 1, (3, 4)).astype(np.float32)
    L = scenes.default_light()
    for nvec, expect_lit in [(L[0], True), (np.array([1.0, -1.0, 0.0]) / math.sqrt(2), False),
                             (-L[0], False)]:
        nrm = np.repeat(np.asarray(nvec, np.float32).reshape(3, 1), 4, axis=1)
        sc = _ndc_scene(W, H, X, Y, [0.5] * 4, color=col, idx=[[0, 1, 3], [0, 3, 2]],
                        normal=nrm, lights=L, shading="deferred")
        o = oracle.render(sc)
        alb = o["gbuf_albedo"][0]
        if expect_lit:
            np.testing.assert_allclose(o["color"][0, :, :, :3], alb, rtol=1e-6, atol=1e-7)
        else:
            assert np.abs(o["color"][0, :, :, :3]).max() <= 1e-7
        np.testing.assert_allclose(np.linalg.norm(o["gbuf_normal"][0], axis=-1), 1.0, rtol=1e-6)


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


# Light sets in which the sum, the last light alone, the first alone and the
# largest term all differ; each holds one light behind the surface, which
# must add nothing (it would subtract without the clamp).
_LIGHT_SETS = [
    [(0, 0, -1), (1, 1, 1), (0, 1, 1), (1, 0, 3)],
    [(1, 1, 1), (0, 0, -1), (0, 1, 1)],
    [(0, 1, 1), (1, 0, 3), (1, 1, 1), (-1, -2, -2)],
]


@pytest.mark.parametrize("shading", ["deferred", "lit"])
@pytest.mark.parametrize("nvec", [(0, 0, 1), (1, 2, 2), (2, -1, 2)])
@pytest.mark.parametrize("which", range(len(_LIGHT_SETS)))
def test_lighting_sums_clamped_terms_over_lights(shading, nvec, which):
    """Several lights: the colour is albedo * sum_l max(0, n.l) with the
    normal and lights fixed by hand (constant over the triangle), the sum
    worked out here in float64.  A back-facing light adds zero.  The lighting
    model is the paper's example fragment shader (material times the dot
    product of normal and light, Sec. 4.1 listing "kernels") clamped at zero
    and summed over the lights, which are the shader-complexity knob of
    Sec. 7.2."""
    W = H = 16
    X = [0, 256 * 16, 0, 256 * 16]
    Y = [0, 0, 256 * 16, 256 * 16]
    alb = np.array([0.8, 0.5, 0.25], np.float32)      # exact in float32
    n = _unit(nvec)
    lights = np.stack([_unit(l) for l in _LIGHT_SETS[which]]).astype(np.float32)
    nrm = np.repeat(n.astype(np.float32).reshape(3, 1), 4, axis=1)
    sc = _ndc_scene(W, H, X, Y, [0.5] * 4, color=np.repeat(alb.reshape(3, 1), 4, axis=1),
                    idx=[[0, 1, 3], [0, 3, 2]], normal=nrm, lights=lights, shading=shading)
    o = oracle.render(sc)
    terms = [max(0.0, float(n @ l.astype(np.float64))) for l in lights]
    assert min(float(n @ l.astype(np.float64)) for l in lights) < -0.1   # one light behind
    expect = alb.astype(np.float64) * sum(terms)
    assert (o["primid"][0] >= 0).all()
    np.testing.assert_allclose(o["color"][0, :, :, :3], np.broadcast_to(expect, (H, W, 3)),
                               rtol=2e-6, atol=0)
    np.testing.assert_array_equal(o["color"][0, :, :, 3], 1.0)
    # the alternatives a mistake would produce are far away
    for wrong in (terms[-1], terms[0], max(terms)):
        assert abs(wrong - sum(terms)) > 0.1


def test_forward_lit_equals_deferred_colour():
    """Forward-lit shading lights the same unit normal and albedo in the
    fragment shader as the deferred pass does from the G-buffer, so the two
    colours agree bit for bit on a random scene with several lights."""
    sc = scenes.micro(num_tris=3000, width=48, height=40, seed=11, num_lights=5)
    d = oracle.render(sc)
    f = oracle.render(SimpleNamespace(**{**vars(sc), "shading": "lit"}), want_gbuf=False)
    np.testing.assert_array_equal(d["primid"], f["primid"])
    np.testing.assert_array_equal(d["color"], f["color"])


# ---------------------------------------------------------------------------
# backward: central differences are exact for the quadratic loss
# ---------------------------------------------------------------------------
def _loss_and_grad(img, tgt, crop):
    y0, y1, x0, x1 = crop
    d = img[:, y0:y1, x0:x1, :3].astype(np.float64) - tgt[:, y0:y1, x0:x1, :3]
    G = np.zeros(img.shape, np.float32)
    G[:, y0:y1, x0:x1, :3] = (2.0 * d).astype(np.float32)
    return float((d * d).sum()), G


def test_backward_matches_central_differences():
    sc = scenes.diffgrid(size=32, num_views=2, nx=8, ny=4, tex_size=8)
    rng = np.random.default_rng(9)
    tgt = rng.uniform(0, 1, (2, 32, 32, 4)).astype(np.float32)
    crop = (8, 24, 8, 24)
    o = oracle.render(sc)
    L0, G = _loss_and_grad(o["color"], tgt, crop)
    gv, gt = oracle.backward(sc, o["primid"], o["bary"], G)
    h = 1e-3
    V = sc.pos.shape[1]
    checked = 0
    for _ in range(24):
        c, v = int(rng.integers(3)), int(rng.integers(V))
        vals = []
        for sgn in (1, -1):
            col = sc.color.copy()
            col[c, v] = np.float32(col[c, v] + sgn * h)
            s2 = SimpleNamespace(**{**vars(sc), "color": col})
            img = oracle.render(s2)["color"]
            vals.append((_loss_and_grad(img, tgt, crop)[0], img))
        fd = (vals[0][0] - vals[1][0]) / (2 * h)
        changed = (vals[0][1] != o["color"]).any(axis=-1).sum()
        bound = 1e-3 * abs(gv[c, v]) + 1e-5 + changed * 3 * 4 * 6e-8 / (2 * h)
        assert abs(fd - gv[c, v]) <= bound, (c, v, fd, gv[c, v])
        checked += gv[c, v] != 0
    for _ in range(24):
        j, i, c = int(rng.integers(8)), int(rng.integers(8)), int(rng.integers(3))
        vals = []
        for sgn in (1, -1):
            tex = sc.texture.copy()
            tex[j, i, c] = np.float32(tex[j, i, c] + sgn * h)
            s2 = SimpleNamespace(**{**vars(sc), "texture": tex})
            img = oracle.render(s2)["color"]
            vals.append((_loss_and_grad(img, tgt, crop)[0], img))
        fd = (vals[0][0] - vals[1][0]) / (2 * h)
        changed = (vals[0][1] != o["color"]).any(axis=-1).sum()
        bound = 1e-3 * abs(gt[j, i, c]) + 1e-5 + changed * 3 * 4 * 6e-8 / (2 * h)
        assert abs(fd - gt[j, i, c]) <= bound, (j, i, c, fd, gt[j, i, c])
        checked += gt[j, i, c] != 0
    assert checked > 10


def test_backward_sum_invariants():
    """Barycentric and bilinear weights each sum to one, so the gradients
    summed over vertices (texels) equal the per-pixel sums of G*T (G*C)."""
    sc = scenes.diffgrid(size=32, num_views=2, nx=8, ny=4, tex_size=8)
    rng = np.random.default_rng(1)
    G = rng.standard_normal((2, 32, 32, 4)).astype(np.float32)
    o = oracle.render(sc)
    gv, gt = oracle.backward(sc, o["primid"], o["bary"], G)
    plain = oracle.render(SimpleNamespace(**{**vars(sc), "shading": "gouraud"}))
    cov = o["primid"] >= 0
    Cint = plain["color"][..., :3].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        T = np.where(Cint != 0, o["color"][..., :3] / Cint, 0.0)
    for c in range(3):
        lhs_v = gv[c].sum()
        rhs_v = (G[..., c].astype(np.float64) * T[..., c])[cov].sum()
        assert abs(lhs_v - rhs_v) <= 1e-5 * np.abs(G[..., c] * T[..., c])[cov].sum()
        lhs_t = gt[..., c].sum()
        rhs_t = (G[..., c].astype(np.float64) * Cint[..., c])[cov].sum()
        assert abs(lhs_t - rhs_t) <= 1e-5 * np.abs(G[..., c] * Cint[..., c])[cov].sum()


# ---------------------------------------------------------------------------
# AssignBin lists
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [0, 4, 8, 16])
def test_assign_bin_vs_bruteforce(B):
    sc = scenes.tiny(seed=21, width=36, height=28, num_tris=14)
    off, tris = oracle.assign_bin(sc, B)
    ref = bf.bins(sc, B)
    nb = len(off) - 1
    for b in range(nb):
        lst = list(tris[off[b]:off[b + 1]])
        assert lst == sorted(lst)
        assert lst == ref.get(b, []), b


# ---------------------------------------------------------------------------
# the oracle on several host threads
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("make", [
    lambda: scenes.tiny(seed=4, width=61, height=47, num_tris=300),
    lambda: scenes.grid(seed=3, width=80, height=45, nx=32, ny=16),
    lambda: scenes.micro(num_tris=20000, width=96, height=64, seed=2),
    lambda: scenes.batch(num_scenes=5, size=48, tmin=50, tmax=500, seed0=8),
])
def test_row_bands_on_threads_equal_single_thread(make):
    """Pixels are computed independently, so rendering bands of rows (or
    scenes) on several threads gives the single-threaded image bit for bit,
    fragment counts included."""
    sc = make()
    a = oracle.render(sc, want_cover=True)
    for threads in (2, 7):
        b = oracle.render(sc, want_cover=True, threads=threads)
        for k, v in a.items():
            if v is not None:
                np.testing.assert_array_equal(b[k], v, err_msg=k)
